// bdc_kernels.hip -- gfx950 kernels of the posterior sampler.
//
// One sweep = forward_propose (mu = P (x) rho from scratch, plus this sweep's
// proposals for every pixel) -> the colour or block-phase passes (footprint
// likelihood deltas, Metropolis decisions, mu commits) -> moments (Welford,
// batched R-hat statistics, per-chain log-posterior partials) -> finalize
// (deterministic reduction of the log-posterior, sweep index + 1).
// The sweep index lives in device memory so a captured sweep replays as is.
#include "bdc_device.h"
#include "bdc_kernels.h"

#include <math.h>

#include <algorithm>

namespace bdc {

namespace {

__device__ inline PixConst load_pc(const float4* pc, int64_t n) {
    // 16-byte records; frames stay below 2^27 pixels, so a 32-bit byte offset
    // from the base suffices
    const float4 u = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(pc) + ((uint32_t)n << 4));
    PixConst p;
    p.c = u.x; p.a2 = u.y; p.L0 = u.z; p.iB = u.w;
    p.ks = fmaxf(p.c, 0.0f);
    p.inv2a = __builtin_amdgcn_rcpf(p.a2);
    p.h0 = __builtin_amdgcn_sqrtf(2.0f * TAIL_T * p.inv2a);
    return p;
}

// Per-pixel constants of the phi window from c and a (see PixConst).
__device__ inline PixConst make_pc(double c, double a) {
    PixConst p;
    const double ks = c > 0.0 ? c : 0.0;
    p.c = (float)c;
    p.a2 = (float)(2.0 * a);
    p.inv2a = (float)(0.5 / a);
    p.ks = (float)ks;
    p.L0 = (float)(2.0 * a * (c - ks) - log(ks + 1.0));
    p.iB = (float)(1.0 / (2.0 * a + 1.0 / (ks + 1.0)));
    p.h0 = (float)sqrt((double)TAIL_T / a);
    return p;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroups go to the XCDs round-robin in dispatch order, and each XCD has
// its own L2.  The chains of one block of a block scan read the same per-pixel
// records, so the block scans map workgroup id to (block, chain) with id mod
// XCDS the XCD: the C chains of block XCDS * q + x are consecutive workgroups
// of XCD x, resident together, and the first chain's record reads leave the
// lines in that XCD's L2 for the others.  Ids past the last block get false
// (the workgroup exits at once).  Grid: xcd_grid(nblk, C).
__device__ inline bool xcd_block(int nblk, int C, int& bi, int& chain) {
    const int64_t id = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;   // dispatch order
    const int x = (int)(id % XCDS);
    const int64_t j = id / XCDS;
    const int64_t bl = XCDS * (j / C) + x;
    chain = (int)(j % C);
    bi = (int)min(bl, (int64_t)nblk);
    return bl < nblk;
}

// Camera value of pixel n (map or scalar).
__device__ inline float cam(const float* p, int per_pixel, int64_t n) { return per_pixel ? p[n] : p[0]; }

// log n! for an integer n >= 0: the log of the exact product below 20 (every
// partial product is exact in double), Stirling's series through the n^-7
// term from 20 on (truncation error below 2e-15).
__device__ inline double log_factorial(int n) {
    if (n < 20) {
        double p = 1.0;
        for (int i = 2; i <= n; ++i) p *= (double)i;
        return log(p);
    }
    const double x = (double)n, ix = rcp_nr(x), ix2 = ix * ix;
    const double corr = ix * (1.0 / 12.0 - ix2 * (1.0 / 360.0 - ix2 * (1.0 / 1260.0 - ix2 * (1.0 / 1680.0))));
    return (x + 0.5) * log(x) - x + 0.91893853320467274178 + corr;   // + log(2 pi) / 2
}

// Sharper read noise than the recurrence takes (a > A_RECUR_MAX, rare): a
// max-shifted log-sum-exp over the (short) window.
__device__ __noinline__ double ell_abs_sharp(double mu, double c, double a, double lnorm, int lo, int hi) {
    const double lmud = log(mu), lf_lo = log_factorial(lo);
    double mx = -INFINITY, lf = lf_lo;                 // lf = log k!
    for (int k = lo; k <= hi; ++k) {
        if (k > lo) lf += log((double)k);
        mx = fmax(mx, -a * (k - c) * (k - c) + k * lmud - lf);
    }
    double s = 0.0;
    lf = lf_lo;
    for (int k = lo; k <= hi; ++k) {
        if (k > lo) lf += log((double)k);
        s += exp(-a * (k - c) * (k - c) + k * lmud - lf - mx);
    }
    return lnorm - mu + mx + log(s);
}

// Absolute log-likelihood of one pixel in double precision (parity output and
// log-posterior trace).  a <= A_RECUR_MAX: Horner from the window top,
//   ell = lnorm - mu + log W_lo + log(1 + sum_{k>lo} W_k / W_lo),
//   log W_lo = -a (lo - c)^2 + lo log mu - log(lo!);
// sharper read noise: ell_abs_sharp.
__device__ inline double ell_abs(float muf, float wv, float gain, float o, float sig) {
    const double c = ((double)wv - (double)o) / (double)gain;
    const double a = (double)gain * (double)gain / (2.0 * (double)sig * (double)sig);
    const double lnorm = -0.5 * log(2.0 * M_PI * (double)sig * (double)sig);
    const double mu = (double)muf;
    if (!(mu > 0.0)) return lnorm - a * c * c;
    const PixConst pc = make_pc(c, a);
    const float lmu = logf(muf);
    const Window win = phi_window(lmu, lmu, pc);
    if (!win.ok) return __builtin_nan("");
    if (a > (double)A_RECUR_MAX) return ell_abs_sharp(mu, c, a, lnorm, win.lo, win.hi);
    const double lmud = log(mu);
    const double qi = exp(2.0 * a);
    double G = mu * exp(-a * (2.0 * (win.hi - 1) + 1.0 - 2.0 * c));
    double acc = 0.0;
#pragma unroll 1
    for (int k = win.hi - 1; k >= win.lo; --k) {
        const double r = G * rcp_nr((double)(k + 1));
        G *= qi;
        acc = fma(r, acc, r);
    }
    const double lo = (double)win.lo;
    const double logw_lo = -a * (lo - c) * (lo - c) + lo * lmud - log_factorial(win.lo);
    return lnorm - mu + logw_lo + log1p(acc);
}

// The same for an EMCCD pixel (bdc_device.h), in double from the raw inputs.
__device__ __noinline__ double ell_abs_emccd(float muf, float wv, float gain, float o, float sig) {
    const double c = ((double)wv - (double)o) / (double)gain;
    const double dw = (double)wv - (double)o, s2 = (double)sig * (double)sig;
    const double lA = -0.5 * log(2.0 * M_PI * s2) - dw * dw / (2.0 * s2);
    const double mu = (double)muf;
    if (!(mu > 0.0)) return lA;
    return emccd_lse(mu, c, lA, -c - log((double)gain)) - mu;
}

template <bool EM>
__device__ inline double ell_abs_cam(const Frame& f, float mu, int64_t n) {
    const float w = f.w[n], G = cam(f.gain, f.cam_per_pixel, n), o = cam(f.offset, f.cam_per_pixel, n),
                sg = cam(f.sigma, f.cam_per_pixel, n);
    if constexpr (EM) return ell_abs_emccd(mu, w, G, o, sg);
    else return ell_abs(mu, w, G, o, sg);
}

// ---------------------------------------------------------------------------
// Frame setup
// ---------------------------------------------------------------------------
__global__ void k_pixel_consts(Frame f, float4* pc, int* bad) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= f.Np) return;
    const float wv = f.w[n];
    const float G = cam(f.gain, f.cam_per_pixel, n);
    const float o = cam(f.offset, f.cam_per_pixel, n);
    const float sg = cam(f.sigma, f.cam_per_pixel, n);
    if (!isfinite(wv) || !isfinite(o) || !isfinite(G) || !isfinite(sg)) { atomicAdd(&bad[0], 1); return; }
    if (!(G > 0.0f) || !(sg > 0.0f)) { atomicAdd(&bad[1], 1); return; }
    const double c = ((double)wv - (double)o) / (double)G;
    if (f.camera == 1) {
        const double dw = (double)wv - (double)o, s2 = (double)sg * (double)sg;
        const double lA = -0.5 * log(2.0 * M_PI * s2) - dw * dw / (2.0 * s2);
        const double lB = c > 0.0 ? -c - log((double)G) : -INFINITY;
        pc[n] = make_float4((float)c, -1.0f, (float)lA, (float)lB);
        return;
    }
    const double a = (double)G * (double)G / (2.0 * (double)sg * (double)sg);
    const PixConst p = make_pc(c, a);
    pc[n] = make_float4(p.c, p.a2, p.L0, p.iB);
}

__global__ void k_init_state(Frame f, State S, const float* rho0, float log_step0, int* bad) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int chain = blockIdx.y;
    if (n >= f.N) return;
    const int64_t i = (int64_t)chain * f.N + n;
    float v;
    if (rho0) {
        v = rho0[i];
        if (!(v > 0.0f) || !isfinite(v)) { atomicAdd(&bad[0], 1); v = 1.0f; }
    } else if (f.sub == 1) {
        const float c = f.pc[n].x;
        const float xi = box_muller(draw(f.key, (uint32_t)n, 0u, (uint32_t)chain, STREAM_INIT));
        v = fmaxf(c, 0.5f) * expf(0.5f * xi);
    } else {
        // a pixel's photon estimate shared by its k x k cells
        const int y = (int)(n / f.W), x = (int)(n % f.W);
        const float c = f.pc[(int64_t)(y / f.sub) * f.Wp + x / f.sub].x;
        const float xi = box_muller(draw(f.key, (uint32_t)n, 0u, (uint32_t)chain, STREAM_INIT));
        v = fmaxf(c, 0.5f) / (float)(f.sub * f.sub) * expf(0.5f * xi);
    }
    S.rho[i] = v;
    S.log_step[i] = log_step0;
}

// ---------------------------------------------------------------------------
// mu = P (x) rho (LDS tile + halo, double accumulation) and this sweep's
// proposals: rho' = rho exp(step xi), step = exp(log_step), xi ~ N(0, 1) from
// stream 0; Hastings + prior terms; log u from stream 1.
// ---------------------------------------------------------------------------
constexpr int FT = 32;   // output tile side

// This sweep's proposal for object cell m of one chain (current value r0).
__device__ inline void propose_cell(const Frame& f, const State& S, const Prior& pr, int64_t m, int chain,
                                    int64_t t, float r0) {
    const int64_t i = (int64_t)chain * f.N + m;
    const float xi = box_muller(draw(f.key, (uint32_t)m, (uint32_t)t, (uint32_t)chain, STREAM_PROPOSAL));
    const float step = expf(S.log_step[i]);
    const float hs = step * xi;                 // log rho' - log rho
    const float rp = r0 * expf(hs);
    float hast = hs;
    if (pr.kind == 1) hast += (pr.a - 1.0f) * hs - pr.b * (rp - r0);
    if (!(rp > 0.0f) || !isfinite(rp)) hast = -INFINITY;
    S.prop_rho[i] = rp;
    S.prop_hast[i] = hast;
    S.prop_logu[i] = logf(u01(draw(f.key, (uint32_t)m, (uint32_t)t, (uint32_t)chain, STREAM_ACCEPT).x));
}

// One FT x FT output tile of one chain.  lds: (FT + 2r)^2 + s^2 floats.
__device__ void forward_tile(const Frame& f, const State& S, const Prior& pr, int propose, int tile, int chain,
                             int64_t t, float* lds) {
    const int r = f.r, s = f.s, TWd = FT + 2 * r;
    float* tl = lds;                                                // rho tile with halo, [TWd][TWd]
    float* sp = lds + TWd * TWd;                                    // PSF, [s][s]
    const int ntx = (f.W + FT - 1) / FT;
    const int ty0 = (tile / ntx) * FT, tx0 = (tile % ntx) * FT;
    const float* rho = S.rho + (int64_t)chain * f.N;
    for (int i = threadIdx.x; i < TWd * TWd; i += WG) {
        const int yy = ty0 - r + i / TWd, xx = tx0 - r + i % TWd;
        tl[i] = (yy >= 0 && yy < f.H && xx >= 0 && xx < f.W) ? rho[(int64_t)yy * f.W + xx] : 0.0f;
    }
    for (int i = threadIdx.x; i < s * s; i += WG) sp[i] = f.psf[i];
    __syncthreads();
    // each thread: four adjacent outputs of one tile row; per PSF row the four
    // share a window of tile values that slides one entry per tap, so each
    // value is loaded and converted once (every output's FMA order and operands
    // are those of a tap-by-tap loop)
    static_assert(FT * FT == 4 * WG, "four outputs per thread");
    const int ly = threadIdx.x / (FT / 4), lx0 = (threadIdx.x % (FT / 4)) * 4;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int dy = -r; dy <= r; ++dy) {
        const float* prow = sp + (dy + r) * s + r;                  // prow[dx]
        const float* trow = tl + (ly - dy + r) * TWd + lx0 + r;     // output k, tap dx: trow[k - dx]
        double w0 = trow[r], w1 = trow[r + 1], w2 = trow[r + 2], w3 = trow[r + 3];
        for (int dx = -r; dx < r; ++dx) {
            const double p = (double)prow[dx];
            acc[0] = fma(p, w0, acc[0]);
            acc[1] = fma(p, w1, acc[1]);
            acc[2] = fma(p, w2, acc[2]);
            acc[3] = fma(p, w3, acc[3]);
            w3 = w2;
            w2 = w1;
            w1 = w0;
            w0 = (double)trow[-dx - 1];
        }
        const double p = (double)prow[r];
        acc[0] = fma(p, w0, acc[0]);
        acc[1] = fma(p, w1, acc[1]);
        acc[2] = fma(p, w2, acc[2]);
        acc[3] = fma(p, w3, acc[3]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int lx = lx0 + k;
        const int y = ty0 + ly, x = tx0 + lx;
        if (y >= f.H || x >= f.W) continue;
        const double accv = acc[k];
        const int64_t m = (int64_t)y * f.W + x;
        const int64_t i = (int64_t)chain * f.N + m;
        S.mu[i] = (float)accv;
        if (propose) propose_cell(f, S, pr, m, chain, t, rho[m]);
    }
}

__global__ void __launch_bounds__(WG) k_forward_propose(Frame f, State S, Prior pr, int propose) {
    extern __shared__ float lds_f[];
    forward_tile(f, S, pr, propose, blockIdx.x, blockIdx.y, *S.t, lds_f);
}

// Finer object lattice (sub = k > 1): pixel n's mean, FP64 accumulation over
// the k^2 phases and the footprint, mu_n = sum_phase sum_d T_phase[d] rho(cell
// of that phase in pixel n - d).
__global__ void __launch_bounds__(WG) k_forward_sub(Frame f, State S) {
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int chain = blockIdx.y;
    if (n >= f.Np) return;
    const int k = f.sub, s = f.s, r = f.r;
    const int py = (int)(n / f.Wp), px = (int)(n % f.Wp);
    const float* rho = S.rho + (int64_t)chain * f.N;
    double acc = 0.0;
    for (int ph = 0; ph < k * k; ++ph) {
        const float* T = f.psf + (int64_t)ph * s * s;
        const int a = ph / k, b = ph % k;
        for (int dy = -r; dy <= r; ++dy) {
            const int qy = py - dy;
            if (qy < 0 || qy >= f.Hp) continue;
            for (int dx = -r; dx <= r; ++dx) {
                const int qx = px - dx;
                if (qx < 0 || qx >= f.Wp) continue;
                acc = fma((double)T[(dy + r) * s + dx + r], (double)rho[(int64_t)(qy * k + a) * f.W + qx * k + b], acc);
            }
        }
    }
    S.mu[(int64_t)chain * f.Np + n] = (float)acc;
}

// This sweep's proposals for every object cell (sub > 1).
__global__ void __launch_bounds__(WG) k_propose_sub(Frame f, State S, Prior pr) {
    const int64_t m = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int chain = blockIdx.y;
    if (m >= f.N) return;
    propose_cell(f, S, pr, m, chain, *S.t, S.rho[(int64_t)chain * f.N + m]);
}

// Decision shared by both scans: accept iff Delta finite and log u < Delta;
// commits rho, adapts the step during burn-in, counts, records for parity.
// hast, logu, rp: this pixel's Hastings + prior term, log u and proposal
// (loaded ahead by the caller, off the decision's critical path).
__device__ inline bool decide_commit(const Frame& f, const State& S, int chain, int64_t m, int64_t t, int burn_in,
                                     double tot, bool writer, float hast, float logu, float rp, float* dbg_delta,
                                     uint8_t* dbg_acc) {
    const int64_t i = (int64_t)chain * f.N + m;
    const double delta = tot + (double)hast;
    const bool acc = isfinite(delta) && ((double)logu < delta);
    if (writer) {
        if (acc) {
            S.rho[i] = rp;
            atomicAdd(&S.accepts[chain], 1ull);
        }
        if (t < burn_in) {
            const float gain = exp2f(-0.6f * log2f((float)t + 1.0f));
            S.log_step[i] += gain * ((acc ? 1.0f : 0.0f) - 0.44f);
        }
        if (dbg_delta) dbg_delta[i] = (float)delta;
        if (dbg_acc) dbg_acc[i] = acc ? 1 : 0;
    }
    return acc;
}

__device__ inline bool decide_and_commit(const Frame& f, const State& S, int chain, int64_t m, int64_t t,
                                         int burn_in, double tot, bool writer,
                                         float* dbg_delta, uint8_t* dbg_acc) {
    const int64_t i = (int64_t)chain * f.N + m;
    return decide_commit(f, S, chain, m, t, burn_in, tot, writer, S.prop_hast[i], S.prop_logu[i], S.prop_rho[i],
                         dbg_delta, dbg_acc);
}

// ---------------------------------------------------------------------------
// Pixel-chromatic pass: one colour (cy, cx) of the s x s colouring; one
// workgroup per (active pixel, chain); footprint spread over the workgroup.
// ---------------------------------------------------------------------------
__device__ inline void count_work(unsigned long long* ctr, int terms, int evals) {
    unsigned long long t = (unsigned long long)terms, e = (unsigned long long)evals;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        t += __shfl_xor(t, off, 64);
        e += __shfl_xor(e, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&ctr[0], t);
        atomicAdd(&ctr[1], e);
    }
}

template <bool EM>
__global__ void __launch_bounds__(WG) k_colour_pass(Frame f, State S, int burn_in, const double* inv_tab,
                                                    int cy, int cx, float* dbg_delta, uint8_t* dbg_acc) {
    __shared__ double s_red[WG / 64];
    __shared__ int s_acc;
    const int s = f.s, r = f.r, F = s * s;
    const int ncol = (f.W - cx + s - 1) / s;
    const int y = cy + s * (blockIdx.x / ncol), x = cx + s * (blockIdx.x % ncol);
    const int chain = blockIdx.y;
    const int64_t m = (int64_t)y * f.W + x;
    const int64_t base = (int64_t)chain * f.N;
    const float d = S.prop_rho[base + m] - S.rho[base + m];
    const float* mu = S.mu + base;
    double part = 0.0;
    int nterms = 0, nevals = 0;
    for (int j = threadIdx.x; j < F; j += WG) {
        const int ny = y + j / s - r, nx = x + j % s - r;
        if (ny < 0 || ny >= f.H || nx < 0 || nx >= f.W) continue;
        const int64_t n = (int64_t)ny * f.W + nx;
        part += delta_pix<EM>(mu[n], d * f.psf[j], load_pc(f.pc, n), inv_tab, nterms);
        ++nevals;
    }
    count_work(S.counters, nterms, nevals);
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
    __syncthreads();
    const int64_t t = *S.t;
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < WG / 64; ++w) tot += s_red[w];
        s_acc = decide_and_commit(f, S, chain, m, t, burn_in, tot, true, dbg_delta, dbg_acc) ? 1 : 0;
    }
    __syncthreads();
    if (s_acc) {
        float* muw = S.mu + base;
        for (int j = threadIdx.x; j < F; j += WG) {
            const int ny = y + j / s - r, nx = x + j % s - r;
            if (ny < 0 || ny >= f.H || nx < 0 || nx >= f.W) continue;
            muw[(int64_t)ny * f.W + nx] += d * f.psf[j];
        }
    }
}

// Pixel-chromatic pass over a finer object lattice (sub = k > 1): the cells of
// one phase (a, b) in the pixels (cy + s i, cx + s j); cell m's footprint is
// the s x s pixels around its own with weights T_phase.
template <bool EM>
__global__ void __launch_bounds__(WG) k_colour_pass_sub(Frame f, State S, int burn_in, const double* inv_tab,
                                                        int phase, int cy, int cx, float* dbg_delta,
                                                        uint8_t* dbg_acc) {
    __shared__ double s_red[WG / 64];
    __shared__ int s_acc;
    const int s = f.s, r = f.r, F = s * s, k = f.sub;
    const int ncol = (f.Wp - cx + s - 1) / s;
    const int py = cy + s * (blockIdx.x / ncol), px = cx + s * (blockIdx.x % ncol);
    const int chain = blockIdx.y;
    const int64_t m = (int64_t)(py * k + phase / k) * f.W + (px * k + phase % k);
    const int64_t base = (int64_t)chain * f.N, pbase = (int64_t)chain * f.Np;
    const float* T = f.psf + (int64_t)phase * F;
    const float d = S.prop_rho[base + m] - S.rho[base + m];
    const float* mu = S.mu + pbase;
    double part = 0.0;
    int nterms = 0, nevals = 0;
    for (int j = threadIdx.x; j < F; j += WG) {
        const int ny = py + j / s - r, nx = px + j % s - r;
        if (ny < 0 || ny >= f.Hp || nx < 0 || nx >= f.Wp) continue;
        const int64_t n = (int64_t)ny * f.Wp + nx;
        part += delta_pix<EM>(mu[n], d * T[j], load_pc(f.pc, n), inv_tab, nterms);
        ++nevals;
    }
    count_work(S.counters, nterms, nevals);
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
    __syncthreads();
    const int64_t t = *S.t;
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < WG / 64; ++w) tot += s_red[w];
        s_acc = decide_and_commit(f, S, chain, m, t, burn_in, tot, true, dbg_delta, dbg_acc) ? 1 : 0;
    }
    __syncthreads();
    if (s_acc) {
        float* muw = S.mu + pbase;
        for (int j = threadIdx.x; j < F; j += WG) {
            const int ny = py + j / s - r, nx = px + j % s - r;
            if (ny < 0 || ny >= f.Hp || nx < 0 || nx >= f.Wp) continue;
            muw[(int64_t)ny * f.Wp + nx] += d * T[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Block-phase pass.  The frame is cut into B x B blocks; blocks whose
// (row, col) parities equal the phase are >= B + 1 >= s pixels apart, so their
// footprint regions (block + r halo) are disjoint and each workgroup owns its
// region's mu in LDS for the whole phase, running the s*s intra-block colours
// [k0, k1) in order with workgroup barriers only.
// ---------------------------------------------------------------------------
constexpr int MAX_ACT = 16;   // active pixels per colour per block (B <= 4 s)

// Divergence control.  A wave's phi-term loop runs as long as its longest
// window, and a pixel's window length is set mostly by a per-pixel constant,
// the half-width h0 = sqrt(T / a) of its read noise.  With one active pixel
// per colour (B <= s, the usual block), every wave sorts its own footprint
// evaluations by the class floor(h0) (a counting sort in wave-private LDS, no
// workgroup barrier) and its lanes take them in that order, so the 64 windows
// evaluated together have nearly the same length.
constexpr int NCLS = 16;           // window classes
constexpr int SORT_MAX_F = 4 * WG; // footprints up to 32 x 32 take the sorted path
constexpr int WAVES = WG / 64;

struct WaveSort {                  // per-wave scratch in LDS
    int hist[NCLS];
    int base[NCLS];
    int count;
    uint16_t order[SORT_MAX_F / WAVES];
};

// (EMCCD pixels carry no window: their h0 is NaN, class 0)
__device__ inline int window_class(float h0) { return h0 >= 0.0f ? min(NCLS - 1, (int)h0) : 0; }

__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for every
// outstanding global load and store of the wave; the block-series pass passes
// no global data between its threads, so its barriers leave global traffic
// (the decision inputs fetched one update ahead, thread 0's commits) in flight.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Dirichlet-OTF prior per chunk (Methods, Prior, Eqs. 7-8).  A chunk is one
// B x B block of the block-phase scan (edge chunks smaller); its prior is the
// Dirichlet of x_k = |F_k| / sum_j |F_j| with concentration alpha_k (the
// normalised |OTF| on the chunk's grid, tabulated per chunk shape by the host),
//   F_k = sum_m rho_m exp(-2 pi i (ky y / th + kx x / tw)).
// A move rho_m -> rho_m + d changes every F_k by d w_k(m), w_k(m) =
// exp(-2 pi i (ky y_m / th + kx x_m / tw)), so with p_k = Re(F_k conj(w_k)),
//   |F_k'|^2 = |F_k|^2 (1 + u_k),  u_k = d (2 p_k + d) / |F_k|^2,
// and the change of the log prior is
//   sum_k (alpha_k - 1) log(1 + u_k) / 2  -  (sum_k (alpha_k - 1)) log(S' / S)
// with S = sum_k |F_k|, S' - S = sum_k d (2 p_k + d) / (|F_k'| + |F_k|): both
// sums free of cancellation, so FP32 terms keep their relative accuracy.
// ---------------------------------------------------------------------------
constexpr int DIR_MAX_B = 32;                 // chunk side (B <= s <= 31 with this prior)
constexpr int DIR_Q = (DIR_MAX_B * DIR_MAX_B + WG - 1) / WG;

struct ChunkGeom { int y0, x0, th, tw, shape; };

__device__ inline ChunkGeom chunk_geom(const Frame& f, int ci) {
    const int B = f.dir_B, ncx = (f.W + B - 1) / B;
    const int cy = ci / ncx, cx = ci - cy * ncx;
    ChunkGeom g;
    g.y0 = cy * B;
    g.x0 = cx * B;
    g.th = min(B, f.H - g.y0);
    g.tw = min(B, f.W - g.x0);
    g.shape = (g.th < B ? 2 : 0) + (g.tw < B ? 1 : 0);
    return g;
}

// a - b floor(a / b) for 0 <= a < 2^20, b >= 1 (exact in FP32 arithmetic)
__device__ inline int small_mod(int a, int b, float inv_b) {
    const int q = (int)(((float)a + 0.5f) * inv_b);
    return a - b * q;
}

// LDS of the chunk prior inside a block pass.  The spectrum is kept in FP64:
// a move can nearly cancel a component (|F'| << |F|), and log|F'| then needs
// F' to more digits than FP32 holds.
struct DirLds {
    double *re, *im;                          // [K] per frequency, each owned by one thread
    float* am1;                               // [K] alpha_k - 1
    double2 *th, *tw;                         // (cos, sin)(2 pi j / n), j < th, j < tw
    double* red;                              // [2 * WAVES]
};

__host__ __device__ inline size_t dir_lds_bytes(int B) {
    return (size_t)2 * B * B * sizeof(double) + (size_t)B * B * sizeof(float) + (size_t)2 * B * sizeof(double2) +
           2 * WAVES * sizeof(double) + 16;
}

// One block (index bi among the blocks of phase (py, px)) of one chain.
// lds: block_phase_lds(B, s) bytes (+ dir_lds_bytes(B) with the chunk prior),
// 8-byte aligned.
template <bool DIR, bool EM>
__device__ void block_phase_block(const Frame& f, const State& S, int burn_in, const double* inv_tab, int B,
                                  int py, int px, int bi, int chain, int64_t t, int k0, int k1,
                                  float* dbg_delta, uint8_t* dbg_acc, double* lds_d) {
    const int s = f.s, r = f.r, F = s * s;
    const int RW = B + 2 * r;
    double* s_inv = lds_d;                                   // [INV_TABLE]
    double* s_red = s_inv + INV_TABLE;                       // [MAX_ACT][WG/64]
    float* s_psf = (float*)(s_red + MAX_ACT * (WG / 64));   // [F]
    float* s_mu = s_psf + F;                                 // [RW*RW], -1 outside the frame
    uint16_t* s_off = (uint16_t*)(s_mu + RW * RW);           // [F]: (dy + r) | (dx + r) << 8
    uint8_t* s_cls = (uint8_t*)(s_off + F);                  // [RW*RW] window class
    __shared__ float s_d[MAX_ACT];                           // rho' - rho of the colour's pixels
    __shared__ WaveSort s_ws[WAVES];
    DirLds dl;
    if (DIR) {
        uintptr_t a = reinterpret_cast<uintptr_t>(s_cls + RW * RW);
        a = (a + 15) & ~(uintptr_t)15;
        dl.red = reinterpret_cast<double*>(a);
        dl.th = reinterpret_cast<double2*>(dl.red + 2 * WAVES);
        dl.tw = dl.th + B;
        dl.re = reinterpret_cast<double*>(dl.tw + B);
        dl.im = dl.re + B * B;
        dl.am1 = reinterpret_cast<float*>(dl.im + B * B);
    }

    const int nbx = (f.W + B - 1) / B;
    const int nbx_p = (nbx - px + 1) / 2;
    const int by = py + 2 * (bi / nbx_p), bx = px + 2 * (bi % nbx_p);
    const int by0 = by * B, bx0 = bx * B;
    const int bh = min(B, f.H - by0), bw = min(B, f.W - bx0);
    const int64_t base = (int64_t)chain * f.N;
    const int ry0 = by0 - r, rx0 = bx0 - r;
    const bool sorted = F <= SORT_MAX_F;

    for (int i = threadIdx.x; i < INV_TABLE; i += WG) s_inv[i] = inv_tab[i];
    for (int j = threadIdx.x; j < F; j += WG) {
        s_psf[j] = f.psf[j];
        s_off[j] = (uint16_t)((j / s) | ((j % s) << 8));
    }
    for (int i = threadIdx.x; i < RW * RW; i += WG) {
        const int yy = ry0 + i / RW, xx = rx0 + i % RW;
        const bool in = yy >= 0 && yy < f.H && xx >= 0 && xx < f.W;
        const int64_t n = (int64_t)yy * f.W + xx;
        s_mu[i] = in ? S.mu[base + n] : -1.0f;
        if (sorted)
            s_cls[i] = in ? (uint8_t)window_class(__builtin_amdgcn_sqrtf(2.0f * TAIL_T / f.pc[n].y)) : 0;
    }
    // chunk prior: this block's spectrum (computed from rho before the pass),
    // per-frequency data owned by thread j % WG, the modulus sum S, twiddles
    double dS_tot = 0.0;
    int dK = 0;
    float inv_bh = 0.0f, inv_bw = 0.0f;
    int jy[DIR_Q], jx[DIR_Q];
    if (DIR) {
        dK = bh * bw;
        inv_bh = 1.0f / (float)bh;
        inv_bw = 1.0f / (float)bw;
        const int shape = (bh < B ? 2 : 0) + (bw < B ? 1 : 0);
        const float* am = f.dir_am1 + (size_t)shape * B * B;
        double sab = 0.0;
#pragma unroll
        for (int q = 0; q < DIR_Q; ++q) {
            const int j = threadIdx.x + q * WG;
            jy[q] = j < dK ? j / bw : 0;
            jx[q] = j < dK ? j - (j / bw) * bw : 0;
            if (j < dK) {
                const double2 F = f.dir_F[base + (int64_t)(by0 + jy[q]) * f.W + (bx0 + jx[q])];
                dl.re[j] = F.x;
                dl.im[j] = F.y;
                dl.am1[j] = am[j];
                sab += sqrt(F.x * F.x + F.y * F.y);
            }
        }
        for (int j = threadIdx.x; j < bh; j += WG) {
            double sn, cs;
            sincospi(2.0 * j / bh, &sn, &cs);
            dl.th[j] = make_double2(cs, sn);
        }
        for (int j = threadIdx.x; j < bw; j += WG) {
            double sn, cs;
            sincospi(2.0 * j / bw, &sn, &cs);
            dl.tw[j] = make_double2(cs, sn);
        }
        sab = wave_sum(sab);
        if ((threadIdx.x & 63) == 0) dl.red[threadIdx.x >> 6] = sab;
        __syncthreads();
        for (int w = 0; w < WAVES; ++w) dS_tot += dl.red[w];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    WaveSort& ws = s_ws[wave];
    int nterms = 0, nevals = 0;
    double dwr[DIR_Q], dwi[DIR_Q];                             // this update's twiddles (chunk prior)

    for (int k = k0; k < k1; ++k) {
        const int ky = k / s, kx = k - (k / s) * s;
        const int nay = bh > ky ? (bh - 1 - ky) / s + 1 : 0;
        const int nax = bw > kx ? (bw - 1 - kx) / s + 1 : 0;
        const int nact = nay * nax;
        if (nact == 0) continue;                              // uniform over the workgroup
        float pre_hast = 0.0f, pre_logu = 0.0f, pre_rp = 0.0f;   // the single pixel's decision inputs
        if (nact == 1 && sorted) {
            const int ly = ky, lx = kx;
            const int64_t m = (int64_t)(by0 + ly) * f.W + (bx0 + lx);
            pre_rp = S.prop_rho[base + m];
            pre_hast = S.prop_hast[base + m];
            pre_logu = S.prop_logu[base + m];
            const float d = pre_rp - S.rho[base + m];
            if (threadIdx.x == 0) s_d[0] = d;
            const int rbase = ly * RW + lx;
            // counting sort of this wave's evaluations by window class
            if (lane < NCLS) ws.hist[lane] = 0;
            wave_fence();
            int key[SORT_MAX_F / WG], rank[SORT_MAX_F / WG];
#pragma unroll
            for (int q = 0; q < SORT_MAX_F / WG; ++q) {
                const int j = threadIdx.x + q * WG;
                key[q] = -1;
                rank[q] = 0;
                if (j < F) {
                    const int o = s_off[j];
                    const int ri = rbase + (o & 0xFF) * RW + (o >> 8);
                    if (s_mu[ri] >= 0.0f) {
                        key[q] = s_cls[ri];
                        rank[q] = atomicAdd(&ws.hist[key[q]], 1);
                    }
                }
            }
            wave_fence();
            if (lane < NCLS) {
                int b = 0;
                for (int c = 0; c < lane; ++c) b += ws.hist[c];
                ws.base[lane] = b;
                if (lane == NCLS - 1) ws.count = b + ws.hist[NCLS - 1];
            }
            wave_fence();
#pragma unroll
            for (int q = 0; q < SORT_MAX_F / WG; ++q)
                if (key[q] >= 0) ws.order[ws.base[key[q]] + rank[q]] = (uint16_t)(threadIdx.x + q * WG);
            wave_fence();
            const int V = ws.count;
            double part = 0.0;
            for (int p = lane; p < V; p += 64) {
                const int j = ws.order[p];
                const int o = s_off[j], oy = o & 0xFF, ox = o >> 8;
                const float muv = s_mu[rbase + oy * RW + ox];
                const int64_t n = m + (int64_t)(oy - r) * f.W + (ox - r);
                part += delta_pix<EM>(muv, d * s_psf[j], load_pc(f.pc, n), s_inv, nterms);
                ++nevals;
            }
            part = wave_sum(part);
            if (lane == 0) s_red[wave] = part;
            if (DIR) {
                double tsum = 0.0, dsum = 0.0;
#pragma unroll
                for (int q = 0; q < DIR_Q; ++q) {
                    const int j = threadIdx.x + q * WG;
                    dwr[q] = 0.0;
                    dwi[q] = 0.0;
                    if (j < dK) {
                        const double2 cy = dl.th[small_mod(jy[q] * ly, bh, inv_bh)];
                        const double2 cx = dl.tw[small_mod(jx[q] * lx, bw, inv_bw)];
                        const double wr = cy.x * cx.x - cy.y * cx.y;
                        const double wi = -(cy.y * cx.x + cy.x * cx.y);
                        dwr[q] = wr;
                        dwi[q] = wi;
                        const double re = dl.re[j], im = dl.im[j], dd = (double)d;
                        const double n2 = re * re + im * im;
                        const double re1 = fma(dd, wr, re), im1 = fma(dd, wi, im);
                        const double n21 = re1 * re1 + im1 * im1;
                        // |F'|^2 - |F|^2 without cancellation for small moves;
                        // the ratio itself when the component shrinks a lot
                        const double num = dd * (2.0 * (re * wr + im * wi) + dd);
                        const float lr = num > -0.5 * n2 ? log1p_k((float)(num / n2)) : fast_ln((float)(n21 / n2));
                        tsum += (double)(dl.am1[j] * 0.5f * lr);
                        dsum += num / (double)(__builtin_amdgcn_sqrtf((float)n21) + __builtin_amdgcn_sqrtf((float)n2));
                    }
                }
                tsum = wave_sum(tsum);
                dsum = wave_sum(dsum);
                if (lane == 0) {
                    dl.red[wave] = tsum;
                    dl.red[WAVES + wave] = dsum;
                }
            }
        } else {
            for (int a = 0; a < nact; ++a) {
                const int ly = ky + s * (a / nax), lx = kx + s * (a % nax);
                const int64_t m = (int64_t)(by0 + ly) * f.W + (bx0 + lx);
                // rho_m is read before any commit of this colour (the barrier below
                // orders the reads before thread 0 overwrites it)
                const float d = S.prop_rho[base + m] - S.rho[base + m];
                if (threadIdx.x == 0) s_d[a] = d;
                const int rbase = ly * RW + lx;                   // footprint origin in the region
                double part = 0.0;
                for (int j = threadIdx.x; j < F; j += WG) {
                    const int o = s_off[j], oy = o & 0xFF, ox = o >> 8;
                    const float muv = s_mu[rbase + oy * RW + ox];
                    if (muv < 0.0f) continue;                     // outside the frame
                    const int64_t n = m + (int64_t)(oy - r) * f.W + (ox - r);
                    part += delta_pix<EM>(muv, d * s_psf[j], load_pc(f.pc, n), s_inv, nterms);
                    ++nevals;
                }
                part = wave_sum(part);
                if ((threadIdx.x & 63) == 0) s_red[a * (WG / 64) + wave] = part;
            }
        }
        __syncthreads();
        for (int a = 0; a < nact; ++a) {
            const int ly = ky + s * (a / nax), lx = kx + s * (a % nax);
            const int64_t m = (int64_t)(by0 + ly) * f.W + (bx0 + lx);
            double tot = 0.0;
            for (int w = 0; w < WG / 64; ++w) tot += s_red[a * (WG / 64) + w];
            double dS = 0.0;
            if (DIR) {
                double tp = 0.0;
                for (int w = 0; w < WAVES; ++w) {
                    tp += dl.red[w];
                    dS += dl.red[WAVES + w];
                }
                // - sum_k (alpha_k - 1) log(S' / S) with sum_k (alpha_k - 1) = 1 - K
                tot += tp + (double)(dK - 1) * log1p(dS / dS_tot);
            }
            const float d = s_d[a];
            const bool acc = (nact == 1 && sorted)
                ? decide_commit(f, S, chain, m, t, burn_in, tot, threadIdx.x == 0, pre_hast, pre_logu, pre_rp,
                                dbg_delta, dbg_acc)
                : decide_and_commit(f, S, chain, m, t, burn_in, tot, threadIdx.x == 0, dbg_delta, dbg_acc);
            if (acc) {
                const int rbase = ly * RW + lx;
                for (int j = threadIdx.x; j < F; j += WG) {
                    const int o = s_off[j];
                    const int ri = rbase + (o & 0xFF) * RW + (o >> 8);
                    const float muv = s_mu[ri];
                    if (muv < 0.0f) continue;
                    s_mu[ri] = muv + d * s_psf[j];
                }
                if (DIR) {
#pragma unroll
                    for (int q = 0; q < DIR_Q; ++q) {
                        const int j = threadIdx.x + q * WG;
                        if (j < dK) {
                            dl.re[j] = fma((double)d, dwr[q], dl.re[j]);
                            dl.im[j] = fma((double)d, dwi[q], dl.im[j]);
                        }
                    }
                    dS_tot += dS;
                }
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < RW * RW; i += WG) {
        const int yy = ry0 + i / RW, xx = rx0 + i % RW;
        if (yy >= 0 && yy < f.H && xx >= 0 && xx < f.W) S.mu[base + (int64_t)yy * f.W + xx] = s_mu[i];
    }
    count_work(S.counters, nterms, nevals);
}

template <bool EM>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5))) k_block_phase(Frame f, State S, int burn_in, const double* inv_tab,
                                                    int B, int py, int px, int k0, int k1,
                                                    float* dbg_delta, uint8_t* dbg_acc, int nblk) {
    extern __shared__ double lds_d[];
    int bi, chain;
    if (!xcd_block(nblk, f.C, bi, chain)) return;
    block_phase_block<false, EM>(f, S, burn_in, inv_tab, B, py, px, bi, chain, *S.t, k0, k1, dbg_delta, dbg_acc,
                                 lds_d);
}

// Block-phase pass over a finer object lattice (sub = k > 1): blocks of B x B
// pixels of one phase (py, px); the block's region of pixel means (block plus
// an r halo) lives in LDS for the whole phase, and the colours [k0, k1) of the
// k^2 s^2 within-block colours (cell phase major, then the pixel position mod
// s, as in the pixel-chromatic scan) run in order, each with one cell per
// active pixel position, the footprint weighted by its phase's table.
// lds: block_phase_sub_lds(B, s, k) bytes.
template <bool EM>
__global__ void __launch_bounds__(WG) k_block_phase_sub(Frame f, State S, int burn_in, const double* inv_tab, int B,
                                                        int py, int px, int k0, int k1, float* dbg_delta,
                                                        uint8_t* dbg_acc, int nblk) {
    extern __shared__ double lds_d[];
    const int s = f.s, r = f.r, F = s * s, k = f.sub, KF = k * k * F;
    const int RW = B + 2 * r;
    double* s_inv = lds_d;                                   // [INV_TABLE]
    double* s_red = s_inv + INV_TABLE;                       // [MAX_ACT][WAVES]
    float* s_psf = (float*)(s_red + MAX_ACT * WAVES);        // [k^2][F]
    float* s_mu = s_psf + KF;                                // [RW*RW], -1 outside the frame
    uint16_t* s_off = (uint16_t*)(s_mu + RW * RW);           // [F]: (dy + r) | (dx + r) << 8
    __shared__ float s_d[MAX_ACT];
    int bi, chain;
    if (!xcd_block(nblk, f.C, bi, chain)) return;
    const int nbx = (f.Wp + B - 1) / B;
    const int nbx_p = (nbx - px + 1) / 2;
    const int by = py + 2 * (bi / nbx_p), bx = px + 2 * (bi % nbx_p);
    const int by0 = by * B, bx0 = bx * B;
    const int bh = min(B, f.Hp - by0), bw = min(B, f.Wp - bx0);
    const int64_t base = (int64_t)chain * f.N, pbase = (int64_t)chain * f.Np;
    const int ry0 = by0 - r, rx0 = bx0 - r;
    const int64_t t = *S.t;
    const int wave = threadIdx.x >> 6;

    for (int i = threadIdx.x; i < INV_TABLE; i += WG) s_inv[i] = inv_tab[i];
    for (int j = threadIdx.x; j < KF; j += WG) s_psf[j] = f.psf[j];
    for (int j = threadIdx.x; j < F; j += WG) s_off[j] = (uint16_t)((j / s) | ((j % s) << 8));
    for (int i = threadIdx.x; i < RW * RW; i += WG) {
        const int yy = ry0 + i / RW, xx = rx0 + i % RW;
        const bool in = yy >= 0 && yy < f.Hp && xx >= 0 && xx < f.Wp;
        s_mu[i] = in ? S.mu[pbase + (int64_t)yy * f.Wp + xx] : -1.0f;
    }
    __syncthreads();
    int nterms = 0, nevals = 0;
    for (int c = k0; c < k1; ++c) {
        const int ph = c / F, kk = c - ph * F;
        const int ky = kk / s, kx = kk - (kk / s) * s;
        const int nay = bh > ky ? (bh - 1 - ky) / s + 1 : 0;
        const int nax = bw > kx ? (bw - 1 - kx) / s + 1 : 0;
        const int nact = nay * nax;
        if (nact == 0) continue;                              // uniform over the workgroup
        const float* T = s_psf + ph * F;
        for (int a = 0; a < nact; ++a) {
            const int ly = ky + s * (a / nax), lx = kx + s * (a % nax);
            const int64_t m = (int64_t)((by0 + ly) * k + ph / k) * f.W + ((bx0 + lx) * k + ph % k);
            // rho_m is read before any commit of this colour (the barrier below
            // orders the reads before thread 0 overwrites it)
            const float d = S.prop_rho[base + m] - S.rho[base + m];
            if (threadIdx.x == 0) s_d[a] = d;
            const int rbase = ly * RW + lx;                   // footprint origin in the region
            double part = 0.0;
            for (int j = threadIdx.x; j < F; j += WG) {
                const int o = s_off[j], oy = o & 0xFF, ox = o >> 8;
                const float muv = s_mu[rbase + oy * RW + ox];
                if (muv < 0.0f) continue;                     // outside the frame
                const int64_t n = (int64_t)(by0 + ly + oy - r) * f.Wp + (bx0 + lx + ox - r);
                part += delta_pix<EM>(muv, d * T[j], load_pc(f.pc, n), s_inv, nterms);
                ++nevals;
            }
            part = wave_sum(part);
            if ((threadIdx.x & 63) == 0) s_red[a * WAVES + wave] = part;
        }
        __syncthreads();
        for (int a = 0; a < nact; ++a) {
            const int ly = ky + s * (a / nax), lx = kx + s * (a % nax);
            const int64_t m = (int64_t)((by0 + ly) * k + ph / k) * f.W + ((bx0 + lx) * k + ph % k);
            double tot = 0.0;
            for (int w = 0; w < WAVES; ++w) tot += s_red[a * WAVES + w];
            const float d = s_d[a];
            if (decide_and_commit(f, S, chain, m, t, burn_in, tot, threadIdx.x == 0, dbg_delta, dbg_acc)) {
                const int rbase = ly * RW + lx;
                for (int j = threadIdx.x; j < F; j += WG) {
                    const int o = s_off[j];
                    const int ri = rbase + (o & 0xFF) * RW + (o >> 8);
                    const float muv = s_mu[ri];
                    if (muv < 0.0f) continue;
                    s_mu[ri] = muv + d * T[j];
                }
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < RW * RW; i += WG) {
        const int yy = ry0 + i / RW, xx = rx0 + i % RW;
        if (yy >= 0 && yy < f.Hp && xx >= 0 && xx < f.Wp) S.mu[pbase + (int64_t)yy * f.Wp + xx] = s_mu[i];
    }
    count_work(S.counters, nterms, nevals);
}

// The block-phase pass with the Dirichlet-OTF prior per chunk (B <= s <= 31).
template <bool EM>
__global__ void __launch_bounds__(WG) k_block_phase_dir(Frame f, State S, int burn_in, const double* inv_tab,
                                                        int B, int py, int px, int k0, int k1,
                                                        float* dbg_delta, uint8_t* dbg_acc, int nblk) {
    extern __shared__ double lds_d[];
    int bi, chain;
    if (!xcd_block(nblk, f.C, bi, chain)) return;
    block_phase_block<true, EM>(f, S, burn_in, inv_tab, B, py, px, bi, chain, *S.t, k0, k1, dbg_delta, dbg_acc,
                                lds_d);
}

// Every chunk's spectrum (MODE 0: into f.dir_F) or log prior (MODE 1: into
// M.dir_part) for one chain: DFT sums in FP64, rows then columns.  One
// workgroup per (chunk, chain).  LDS: chunk_fourier_lds(B) bytes.
template <int MODE>
__global__ void __launch_bounds__(WG) k_chunk_fourier(Frame f, State S, MomentBufs M) {
    extern __shared__ double lds_c[];
    const int ci = blockIdx.x, chain = blockIdx.y;
    const ChunkGeom g = chunk_geom(f, ci);
    const int K = g.th * g.tw;
    double* r = lds_c;                         // [K] rho, later |F|
    double* gre = r + K;                       // [K] row transforms
    double* gim = gre + K;
    double* cth = gim + K;                     // cos, sin (2 pi j / th), (2 pi j / tw)
    double* sth = cth + g.th;
    double* ctw = sth + g.th;
    double* stw = ctw + g.tw;
    double* red = stw + g.tw;                  // [WAVES]
    const int64_t base = (int64_t)chain * f.N;
    for (int i = threadIdx.x; i < K; i += WG) {
        const int y = i / g.tw, x = i - (i / g.tw) * g.tw;
        r[i] = (double)S.rho[base + (int64_t)(g.y0 + y) * f.W + (g.x0 + x)];
    }
    for (int j = threadIdx.x; j < g.th; j += WG) sincospi(2.0 * j / g.th, &sth[j], &cth[j]);
    for (int j = threadIdx.x; j < g.tw; j += WG) sincospi(2.0 * j / g.tw, &stw[j], &ctw[j]);
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += WG) {
        const int y = i / g.tw, kx = i - (i / g.tw) * g.tw;
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int x = 0; x < g.tw; ++x) {
            const double v = r[y * g.tw + x];
            re = fma(v, ctw[idx], re);
            im = fma(-v, stw[idx], im);
            idx += kx;
            if (idx >= g.tw) idx -= g.tw;
        }
        gre[i] = re;
        gim[i] = im;
    }
    __syncthreads();
    double sab = 0.0;
    for (int i = threadIdx.x; i < K; i += WG) {
        const int ky = i / g.tw, kx = i - (i / g.tw) * g.tw;
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int y = 0; y < g.th; ++y) {
            const double a = gre[y * g.tw + kx], b = gim[y * g.tw + kx], cs = cth[idx], sn = sth[idx];
            re += a * cs + b * sn;
            im += b * cs - a * sn;
            idx += ky;
            if (idx >= g.th) idx -= g.th;
        }
        if (MODE == 0) {
            f.dir_F[base + (int64_t)(g.y0 + ky) * f.W + (g.x0 + kx)] = make_double2(re, im);
        } else {
            r[i] = sqrt(re * re + im * im);
            sab += r[i];
        }
    }
    if (MODE == 0) return;
    sab = wave_sum(sab);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sab;
    __syncthreads();
    double Ssum = 0.0;
    for (int w = 0; w < WAVES; ++w) Ssum += red[w];
    __syncthreads();
    const float* am = f.dir_am1 + (size_t)g.shape * f.dir_B * f.dir_B;
    double lp = 0.0;
    for (int i = threadIdx.x; i < K; i += WG) lp += (double)am[i] * log(r[i] / Ssum);
    lp = wave_sum(lp);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = f.dir_const[g.shape];
        for (int w = 0; w < WAVES; ++w) t += red[w];
        M.dir_part[(int64_t)ci * f.C + chain] = t;
    }
}

// ---------------------------------------------------------------------------
// Block-series pass: the block-phase scan for blocks with one active pixel per
// colour (B <= s), where each footprint pixel's likelihood change comes from a
// cached local series (series_at) whenever the move stays inside the series'
// radius, and from delta_ell otherwise.
//
// LDS ring: the s region rows that the footprints of one block row cover
// (region row y in slot y mod s), two 16-byte records per pixel:
//   st = (mu, D, R, -): the current mean (< 0 outside the frame), its
//   displacement from the series anchor mu - D, and the series radius;
//   b = (b1..b4), the series coefficients at the anchor.
// Moving to the next block row writes the oldest row back to mu and loads the
// next region row with fresh series.  Each thread holds SER_Q footprint
// entries, in descending PSF weight: the first (q = 0) covers the PSF core,
// where relative moves are large, so direct evaluations fall almost only on
// q = 0 and a wave runs delta_ell about once per update.  That evaluation also
// forms the series at mu + d, which the lane installs if the move is accepted
// (|D + d| > R leaves the radius, so the old series is spent).
// Counters: [0] phi terms of direct evaluations, [1] footprint evaluations,
// [2] direct evaluations, [3] series anchored from scratch (series_at: new
// ring rows, rare commits), [4] their phi terms, [5] series re-anchored inside
// a direct evaluation.
// ---------------------------------------------------------------------------
constexpr int SER_Q = 4;                      // footprint entries per thread (F <= SER_Q * WG)

__device__ inline void count_work6(unsigned long long* ctr, int terms, int evals, int direct, int anchors,
                                   int anchor_terms, int fused) {
    unsigned long long v[6] = {(unsigned long long)terms, (unsigned long long)evals, (unsigned long long)direct,
                               (unsigned long long)anchors, (unsigned long long)anchor_terms, (unsigned long long)fused};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) atomicAdd(&ctr[k], v[k]);
    }
}

// Lane permutations within rows of 16 (data-parallel primitives, no LDS).
template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int2 u = __builtin_bit_cast(int2, v);
    int2 w;
    w.x = __builtin_amdgcn_update_dpp(0, u.x, CTRL, 0xF, 0xF, false);
    w.y = __builtin_amdgcn_update_dpp(0, u.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, w);
}

__device__ inline double readlane_d(double v, int lane) {
    const int2 u = __builtin_bit_cast(int2, v);
    int2 w;
    w.x = __builtin_amdgcn_readlane(u.x, lane);
    w.y = __builtin_amdgcn_readlane(u.y, lane);
    return __builtin_bit_cast(double, w);
}

// Sum over the 64 lanes, the same value in every lane: pairs, quads, half rows
// and rows by DPP, then the four row sums in a fixed order.
__device__ inline double wave_sum_dpp(double v) {
    v += dpp_d<0xB1>(v);      // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);      // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);     // row_half_mirror
    v += dpp_d<0x140>(v);     // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// LDS ring of one block: per region pixel (slot * RW + x), 28 bytes in three
// arrays: A = (D, R, b1, b2), B = (b3, b4), and the series anchor ma; the
// current mean is ma + D.  R < 0 marks pixels outside the frame.
struct Ring {
    float4* A;
    float2* B;
    float* ma;
};

// Load region rows [y0, y0 + n) (block-local, possibly outside the frame) into
// their ring slots with fresh series, spread over the workgroup's NT threads.
template <int NT = WG>
__device__ inline void series_load_rows(const Frame& f, const State& S, int64_t base, int ry0, int rx0, int RW, int y0,
                                        int n, const Ring& ring, int& nterms, int& nanch) {
    for (int i = threadIdx.x; i < n * RW; i += NT) {
        const int y = y0 + i / RW, xx = i - (i / RW) * RW;
        const int gy = ry0 + y, gx = rx0 + xx;
        float4 A = make_float4(0.0f, -1.0f, 0.0f, 0.0f);
        float2 Bv = make_float2(0.0f, 0.0f);
        float mu = -1.0f;
        if (gy >= 0 && gy < f.H && gx >= 0 && gx < f.W) {
            const int64_t pn = (int64_t)gy * f.W + gx;
            mu = S.mu[base + pn];
            const Series sr = series_at(mu, load_pc(f.pc, pn), nterms);
            A = make_float4(0.0f, sr.R, sr.b.x, sr.b.y);
            Bv = make_float2(sr.b.z, sr.b.w);
            ++nanch;
        }
        const int ri = (y % f.s) * RW + xx;
        ring.A[ri] = A;
        ring.B[ri] = Bv;
        ring.ma[ri] = mu;
    }
}

// Write the means of region rows [y0, y0 + n) back to the frame.
template <int NT = WG>
__device__ inline void series_store_rows(const Frame& f, const State& S, int64_t base, int ry0, int rx0, int RW, int y0,
                                         int n, const Ring& ring) {
    for (int i = threadIdx.x; i < n * RW; i += NT) {
        const int y = y0 + i / RW, xx = i - (i / RW) * RW;
        const int gy = ry0 + y, gx = rx0 + xx;
        if (gy >= 0 && gy < f.H && gx >= 0 && gx < f.W) {
            const int ri = (y % f.s) * RW + xx;
            S.mu[base + (int64_t)gy * f.W + gx] = ring.ma[ri] + ring.A[ri].x;
        }
    }
}

__device__ void block_series_block(const Frame& f, const State& S, int burn_in, int B,
                                   int py, int px, int bi, int chain, int64_t t, int k0, int k1, float* dbg_delta,
                                   uint8_t* dbg_acc, double* lds_d) {
    const int s = f.s, r = f.r, F = s * s;
    const int RW = B + 2 * r, NR = s * RW;
    double* s_red = lds_d;                                          // [2][WAVES]
    Ring ring;
    ring.A = reinterpret_cast<float4*>(s_red + 2 * WAVES);          // [NR]
    ring.B = reinterpret_cast<float2*>(ring.A + NR);                // [NR]
    ring.ma = reinterpret_cast<float*>(ring.B + NR);                // [NR]

    const int nbx = (f.W + B - 1) / B;
    const int nbx_p = (nbx - px + 1) / 2;
    const int by = py + 2 * (bi / nbx_p), bx = px + 2 * (bi % nbx_p);
    const int by0 = by * B, bx0 = bx * B;
    const int bh = min(B, f.H - by0), bw = min(B, f.W - bx0);
    const int64_t base = (int64_t)chain * f.N;
    const int ry0 = by0 - r, rx0 = bx0 - r;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    // this thread's footprint entries, the heaviest PSF weights first:
    // offsets (oy, ox) packed as oy | ox << 8, and the weight
    int off[SER_Q];
    float pw[SER_Q];
#pragma unroll
    for (int q = 0; q < SER_Q; ++q) {
        const int e = threadIdx.x + q * WG;
        const int j = e < F ? (int)f.psf_order[e] : -1;
        off[q] = j >= 0 ? ((j / s) | ((j % s) << 8)) : -1;
        pw[q] = j >= 0 ? f.psf[j] : 0.0f;
    }
    const int oy0 = off[0] & 0xFF, ox0 = (off[0] >> 8) & 0xFF;
    int nterms = 0, nevals = 0, ndirect = 0, nanch = 0, aterms = 0, nfused = 0;
    // the colours [k0, k1) visit rows ly of the block, columns [lx_lo, lx_hi)
    auto lx_lo = [&](int y) { return max(0, k0 - y * s); };
    auto lx_hi = [&](int y) { return min(bw, k1 - y * s); };
    int ly = k0 / s, lx = lx_lo(ly);
    while (ly < bh && lx >= lx_hi(ly)) { ++ly; lx = lx_lo(ly); }
    if (ly >= bh) {
        count_work6(S.counters, 0, 0, 0, 0, 0, 0);
        return;
    }
    int ly_cur = ly;
    // ring index of each entry at column 0 of the current block row
    int rb[SER_Q];
    auto row_bases = [&](int y) {
        const int slot0 = y % s;
#pragma unroll
        for (int q = 0; q < SER_Q; ++q) {
            const int oy = off[q] & 0xFF, ox = (off[q] >> 8) & 0xFF;
            int slot = slot0 + oy;
            slot = slot >= s ? slot - s : slot;
            rb[q] = off[q] >= 0 ? slot * RW + ox : 0;
        }
    };
    row_bases(ly_cur);
    series_load_rows(f, S, base, ry0, rx0, RW, ly_cur, s, ring, aterms, nanch);
    lds_barrier();
    // inputs of the next update, loaded one update ahead: the decision inputs,
    // and the per-pixel constants of this thread's PSF-core entry (q = 0),
    // where direct evaluations fall
    float n_rp, n_hast, n_logu, n_rho;
    float4 n_pc = make_float4(0.0f, 1.0f, 0.0f, 0.0f);
    auto prefetch = [&](int y, int x) {
        const int64_t i = base + (int64_t)(by0 + y) * f.W + (bx0 + x);
        n_rp = S.prop_rho[i];
        n_hast = S.prop_hast[i];
        n_logu = S.prop_logu[i];
        n_rho = S.rho[i];
        const int gy = by0 + y + oy0 - r, gx = bx0 + x + ox0 - r;
        if (off[0] >= 0 && gy >= 0 && gy < f.H && gx >= 0 && gx < f.W) n_pc = f.pc[(int64_t)gy * f.W + gx];
    };
    prefetch(ly, lx);
    const float gain = t < burn_in ? exp2f(-0.6f * log2f((float)t + 1.0f)) : 0.0f;
    // Commits of rho and of the step adaptation are kept per block row: thread
    // x < bw holds pixel (row, x) and writes it back when the row is done, so
    // no global store is outstanding while a wave waits for its next inputs.
    const bool row_owner = threadIdx.x < bw;
    float row_rho = 0.0f, row_ls = 0.0f;
    bool row_acc = false;
    int row_y = -1;
    unsigned long long n_acc = 0;
    auto row_begin = [&](int y) {
        row_y = y;
        row_acc = false;
        if (row_owner && t < burn_in) row_ls = S.log_step[base + (int64_t)(by0 + y) * f.W + (bx0 + threadIdx.x)];
    };
    auto row_end = [&]() {
        if (row_y < 0 || !row_owner) return;
        const int64_t i = base + (int64_t)(by0 + row_y) * f.W + (bx0 + threadIdx.x);
        if (row_acc) S.rho[i] = row_rho;
        if (t < burn_in) S.log_step[i] = row_ls;
    };
    row_begin(ly);
    int par = 0;
    while (ly < bh) {
        const float rp = n_rp, hast = n_hast, logu = n_logu;
        const float d0 = rp - n_rho;
        const float4 pcv0 = n_pc;
        int nly = ly, nlx = lx + 1;
        while (nly < bh && nlx >= lx_hi(nly)) { ++nly; nlx = lx_lo(nly); }
        if (nly < bh) prefetch(nly, nlx);                           // another pixel: no conflict with this commit
        if (ly != row_y) {
            row_end();
            row_begin(ly);
        }
        if (ly != ly_cur) {
            // rows ly_cur .. ly - 1 retire; their slots take the rows s below
            const int nr = min(ly - ly_cur, s);
            series_store_rows(f, S, base, ry0, rx0, RW, ly_cur, nr, ring);
            lds_barrier();
            series_load_rows(f, S, base, ry0, rx0, RW, ly - nr + s, nr, ring, aterms, nanch);
            ly_cur = ly;
            row_bases(ly);
            lds_barrier();
        }
        const int64_t m = (int64_t)(by0 + ly) * f.W + (bx0 + lx);
        // 1. every entry's records, loads issued together
        int ri[SER_Q];
        float4 Aq[SER_Q];
        float2 Bq[SER_Q];
#pragma unroll
        for (int q = 0; q < SER_Q; ++q) {
            ri[q] = off[q] >= 0 ? rb[q] + lx : 0;
            Aq[q] = ring.A[ri[q]];
            Bq[q] = ring.B[ri[q]];
        }
        const float ma0 = ring.ma[ri[0]];                           // the PSF-core entry may go direct
        // 2. series or direct
        int fast = 0, need = 0;
        float dq[SER_Q];
#pragma unroll
        for (int q = 0; q < SER_Q; ++q) {
            dq[q] = d0 * pw[q];
            if (off[q] >= 0 && Aq[q].y >= 0.0f) {
                ++nevals;
                if (fabsf(Aq[q].x + dq[q]) <= Aq[q].y) fast |= 1 << q;
                else need |= 1 << q;
            }
        }
        double part = 0.0;
        // 3. direct terms first (the critical path).  Each lane's first direct
        // entry runs in one pass over the wave, which keeps its window's
        // recurrence state for the series at mu + d, formed after the decision
        // if the move is accepted; a lane's further direct entries (rare)
        // follow.  The PSF-core entry (q = 0) has its per-pixel record
        // prefetched.
        DirectKeep dk;
        dk.n4 = -1;
        const int rest = need & (need - 1);                         // all but the first
        float mu_s = 0.0f, d_s = 0.0f;
        int ri_s = 0;
        if (need) {
            // the lowest set bit of need: an entry classified direct, so valid
            // and inside the frame
            const int qs = __builtin_ctz((unsigned)need);
            int off_s = off[0];
            float D_s = Aq[0].x;
            d_s = dq[0];
            ri_s = ri[0];
#pragma unroll
            for (int q = 1; q < SER_Q; ++q) {
                if (q == qs) {
                    off_s = off[q];
                    D_s = Aq[q].x;
                    d_s = dq[q];
                    ri_s = ri[q];
                }
            }
            PixConst pcs;
            if (need & 1) {
                mu_s = ma0 + D_s;
                pcs.c = pcv0.x; pcs.a2 = pcv0.y; pcs.L0 = pcv0.z; pcs.iB = pcv0.w;
                pcs.ks = fmaxf(pcs.c, 0.0f);
                pcs.inv2a = __builtin_amdgcn_rcpf(pcs.a2);
                pcs.h0 = __builtin_amdgcn_sqrtf(2.0f * TAIL_T * pcs.inv2a);
            } else {
                mu_s = ring.ma[ri_s] + D_s;
                const int oy = off_s & 0xFF, ox = off_s >> 8;
                pcs = load_pc(f.pc, m + (int64_t)(oy - r) * f.W + (ox - r));
            }
            part += delta_ell_keep(mu_s, d_s, pcs, nterms, dk);
        }
        if (rest) {
#pragma unroll
            for (int q = 1; q < SER_Q; ++q) {
                if ((rest >> q) & 1) {
                    const int oy = off[q] & 0xFF, ox = off[q] >> 8;
                    part += delta_ell_notab(ring.ma[ri[q]] + Aq[q].x, dq[q],
                                            load_pc(f.pc, m + (int64_t)(oy - r) * f.W + (ox - r)), nterms);
                }
            }
        }
        // 4. series terms (this lane's few in FP32: their rounding stays
        // relative to the sum of the terms' magnitudes)
        float fpart = 0.0f;
#pragma unroll
        for (int q = 0; q < SER_Q; ++q)
            if ((fast >> q) & 1) fpart += series_delta(make_float4(Aq[q].z, Aq[q].w, Bq[q].x, Bq[q].y), Aq[q].x, dq[q]);
        part += (double)fpart;
        ndirect += __popc(need);
        part = wave_sum_dpp(part);
        if (lane == 0) s_red[par * WAVES + wave] = part;
        lds_barrier();
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) tot += s_red[par * WAVES + w];
        par ^= 1;
        // the decision (identical in every thread)
        const double delta = tot + (double)hast;
        const bool acc = isfinite(delta) && ((double)logu < delta);
        if (threadIdx.x == lx) {
            if (acc) {
                row_rho = rp;
                row_acc = true;
            }
            row_ls += gain * ((acc ? 1.0f : 0.0f) - 0.44f);
        }
        n_acc += acc ? 1 : 0;
        if (threadIdx.x == 0) {
            if (dbg_delta) dbg_delta[base + m] = (float)delta;
            if (dbg_acc) dbg_acc[base + m] = acc ? 1 : 0;
        }
        if (acc) {
#pragma unroll
            for (int q = 0; q < SER_Q; ++q) {
                if ((fast >> q) & 1) ring.A[ri[q]].x = Aq[q].x + dq[q];
            }
            // direct cases left their series' radius: re-anchor at the new mean
            if (need && d_s != 0.0f) {
                const Series nx = series_kept(dk, mu_s, d_s);
                ring.A[ri_s] = make_float4(0.0f, nx.R, nx.b.x, nx.b.y);
                ring.B[ri_s] = make_float2(nx.b.z, nx.b.w);
                ring.ma[ri_s] = mu_s + d_s;
                ++nfused;
            }
#pragma unroll
            for (int q = 1; q < SER_Q; ++q) {
                if (((rest >> q) & 1) && dq[q] != 0.0f) {
                    const int oy = off[q] & 0xFF, ox = off[q] >> 8;
                    const float mu1 = (ring.ma[ri[q]] + Aq[q].x) + dq[q];
                    const Series sr = series_at(mu1, load_pc(f.pc, m + (int64_t)(oy - r) * f.W + (ox - r)), aterms);
                    ring.A[ri[q]] = make_float4(0.0f, sr.R, sr.b.x, sr.b.y);
                    ring.B[ri[q]] = make_float2(sr.b.z, sr.b.w);
                    ring.ma[ri[q]] = mu1;
                    ++nanch;
                }
            }
            lds_barrier();                                          // commits before the next footprint reads
        }
        ly = nly;
        lx = nlx;
    }
    row_end();
    if (threadIdx.x == 0) atomicAdd(&S.accepts[chain], n_acc);
    series_store_rows(f, S, base, ry0, rx0, RW, ly_cur, s, ring);
    count_work6(S.counters, nterms, nevals, ndirect, nanch, aterms, nfused);
}

__global__ void __launch_bounds__(WG) k_block_series(Frame f, State S, int burn_in, int B,
                                                     int py, int px, int k0, int k1, float* dbg_delta,
                                                     uint8_t* dbg_acc, int nblk) {
    extern __shared__ double lds_d[];
    int bi, chain;
    if (!xcd_block(nblk, f.C, bi, chain)) return;
    block_series_block(f, S, burn_in, B, py, px, bi, chain, *S.t, k0, k1, dbg_delta, dbg_acc, lds_d);
}

// ---------------------------------------------------------------------------
// Block-series pass of the nine-phase scan: one wavefront per block.
//
// Blocks of side B in [(s - 1)/2, s] keep the ring of s region rows at
// s (B + s - 1) pixels, small enough for four workgroups per CU, and one
// wavefront holds a whole footprint (up to 16 entries per lane, entry
// e = lane + 64 q in descending PSF weight), so an update needs no workgroup
// barrier: a wave-wide reduction and in-order LDS suffice.  The footprint
// terms that leave their series' radius (a few dozen per update, spread over
// the PSF's heaviest few hundred entries) are queued in LDS and evaluated in
// one pass, one per lane, whatever lanes own them; the owner, which fetched
// every entry's (c, 2a) one update ahead, queues them with the term, and the
// evaluating lane derives the window constants L0 and iB from them (the
// window bracket holds for whatever (c, a) the summands use).  Terms,
// decisions and commits are those of the block-series pass.
// ---------------------------------------------------------------------------
constexpr int WS_NQ = 16;                       // footprint entries per lane (F <= 1024)
constexpr int WS_QCAP = 48;                     // queued direct terms per update; beyond, the owner lanes

__device__ inline PixConst pc_from(float c, float a2) {
    PixConst pc;
    pc.c = c;
    pc.a2 = a2;
    pc.ks = fmaxf(c, 0.0f);
    const float ik = __builtin_amdgcn_rcpf(pc.ks + 1.0f);
    pc.L0 = a2 * (c - pc.ks) - fast_ln(pc.ks + 1.0f);
    pc.iB = __builtin_amdgcn_rcpf(a2 + ik);
    pc.inv2a = __builtin_amdgcn_rcpf(a2);
    pc.h0 = __builtin_amdgcn_sqrtf(2.0f * TAIL_T * pc.inv2a);
    return pc;
}

__device__ inline int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int NQ>
__device__ void wave_series_block(const Frame& f, const State& S, int burn_in, int B, int py, int px, int bi,
                                  int chain, int64_t t, int k0, int k1, float* dbg_delta, uint8_t* dbg_acc,
                                  double* lds_d) {
    const int s = f.s, r = f.r, F = s * s;
    const int RW = B + 2 * r, NR = s * RW;
    // queue slot WS_QCAP and ring cell NR are write sinks: lanes with nothing
    // to queue or commit write there, so the per-entry steps need no branches
    float4* jobs = reinterpret_cast<float4*>(lds_d);                // [WS_QCAP + 1]: (mu, d, c, 2a)
    int* job_ri = reinterpret_cast<int*>(jobs + WS_QCAP + 1);       // [WS_QCAP + 1]: ring index
    Ring ring;
    ring.A = reinterpret_cast<float4*>(job_ri + WS_QCAP + 1);       // [NR + 1]
    ring.B = reinterpret_cast<float2*>(ring.A + NR + 1);            // [NR + 1]
    ring.ma = reinterpret_cast<float*>(ring.B + NR + 1);            // [NR + 1]

    const int nbx = (f.W + B - 1) / B;
    const int nbx_p = (nbx - px + 2) / 3;
    const int by = py + 3 * (bi / nbx_p), bx = px + 3 * (bi % nbx_p);
    const int by0 = by * B, bx0 = bx * B;
    const int bh = min(B, f.H - by0), bw = min(B, f.W - bx0);
    const int64_t base = (int64_t)chain * f.N;
    const int ry0 = by0 - r, rx0 = bx0 - r;
    const int lane = threadIdx.x;
    if (lane == 0) {
        ring.A[NR] = make_float4(0.0f, -1.0f, 0.0f, 0.0f);          // never inside a radius
        ring.B[NR] = make_float2(0.0f, 0.0f);
        ring.ma[NR] = 0.0f;
    }

    int off[NQ];
    float pw[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = lane + 64 * q;
        const int j = e < F ? (int)f.psf_order[e] : -1;
        off[q] = j >= 0 ? ((j / s) | ((j % s) << 8)) : -1;
        pw[q] = j >= 0 ? f.psf[j] : 0.0f;
    }
    int nterms = 0, nevals = 0, ndirect = 0, nanch = 0, aterms = 0, nfused = 0;
    auto lx_lo = [&](int y) { return max(0, k0 - y * s); };
    auto lx_hi = [&](int y) { return min(bw, k1 - y * s); };
    int ly = k0 / s, lx = lx_lo(ly);
    while (ly < bh && lx >= lx_hi(ly)) { ++ly; lx = lx_lo(ly); }
    if (ly >= bh) {
        count_work6(S.counters, 0, 0, 0, 0, 0, 0);
        return;
    }
    int ly_cur = ly;
    // ring index of each entry at column 0 of the current block row (padding
    // entries: the sink cell, whatever the column)
    int rb[NQ];
    auto row_bases = [&](int y) {
        const int slot0 = y % s;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int oy = off[q] & 0xFF, ox = (off[q] >> 8) & 0xFF;
            int slot = slot0 + oy;
            slot = slot >= s ? slot - s : slot;
            rb[q] = off[q] >= 0 ? slot * RW + ox : NR;
        }
    };
    auto ring_index = [&](int q) { return off[q] >= 0 ? rb[q] + lx : NR; };
    row_bases(ly_cur);
    series_load_rows<64>(f, S, base, ry0, rx0, RW, ly_cur, s, ring, aterms, nanch);
    wave_fence();
    // inputs of the next update, fetched one update ahead: the decision inputs
    // and every entry's (c, 2a), through a buffer resource whose range check
    // turns the reads of entries outside the frame into zeros (such entries
    // have invalid ring records and are never queued)
    float n_rp, n_hast, n_logu, n_rho;
    float2 pcq[NQ];
    const __amdgpu_buffer_rsrc_t pc_rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)f.pc, 0, (int)(f.N * (int64_t)sizeof(float4)), 0x00020000);
    const int row_stride = f.W - s;                                 // so that (oy, ox) -> oy W + ox - r (W + 1)
    (void)row_stride;
    auto prefetch = [&](int y, int x) {
        const int64_t m = (int64_t)(by0 + y) * f.W + (bx0 + x);
        n_rp = S.prop_rho[base + m];
        n_hast = S.prop_hast[base + m];
        n_logu = S.prop_logu[base + m];
        n_rho = S.rho[base + m];
        const int m0 = (int)m - r * (f.W + 1);                      // the footprint's top-left pixel
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int oy = off[q] & 0xFF, ox = (off[q] >> 8) & 0xFF;
            const unsigned byte_off = (unsigned)(m0 + oy * f.W + ox) * (unsigned)sizeof(float4);
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(pc_rsrc, byte_off, 0, 0);
            pcq[q] = __builtin_bit_cast(float2, v);
        }
    };
    prefetch(ly, lx);
    const float gain = t < burn_in ? exp2f(-0.6f * log2f((float)t + 1.0f)) : 0.0f;
    const bool row_owner = lane < bw;
    float row_rho = 0.0f, row_ls = 0.0f;
    bool row_acc = false;
    int row_y = -1;
    unsigned long long n_acc = 0;
    auto row_begin = [&](int y) {
        row_y = y;
        row_acc = false;
        if (row_owner && t < burn_in) row_ls = S.log_step[base + (int64_t)(by0 + y) * f.W + (bx0 + lane)];
    };
    auto row_end = [&]() {
        if (row_y < 0 || !row_owner) return;
        const int64_t i = base + (int64_t)(by0 + row_y) * f.W + (bx0 + lane);
        if (row_acc) S.rho[i] = row_rho;
        if (t < burn_in) S.log_step[i] = row_ls;
    };
    row_begin(ly);
    while (ly < bh) {
        const float rp = n_rp, hast = n_hast, logu = n_logu;
        const float d0 = rp - n_rho;
        int nly = ly, nlx = lx + 1;
        while (nly < bh && nlx >= lx_hi(nly)) { ++nly; nlx = lx_lo(nly); }
        if (ly != row_y) {
            row_end();
            row_begin(ly);
        }
        if (ly != ly_cur) {
            const int nr = min(ly - ly_cur, s);
            series_store_rows<64>(f, S, base, ry0, rx0, RW, ly_cur, nr, ring);
            wave_fence();
            series_load_rows<64>(f, S, base, ry0, rx0, RW, ly - nr + s, nr, ring, aterms, nanch);
            ly_cur = ly;
            row_bases(ly);
            wave_fence();
        }
        const int64_t m = (int64_t)(by0 + ly) * f.W + (bx0 + lx);
        // 1. every entry's record (four entries' loads issued together); its
        //    series term, or its place in the queue of terms outside their
        //    radius, with the (c, 2a) fetched for it
        unsigned fast = 0, over = 0;
        int nq = 0;
        float fpart = 0.0f;
        float Dq[NQ];
#pragma unroll
        for (int g = 0; g < NQ; g += 4) {
            float4 Aq[4];
            float2 Bq[4];
            float maq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ri = ring_index(g + u);
                Aq[u] = ring.A[ri];
                Bq[u] = ring.B[ri];
                maq[u] = ring.ma[ri];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = g + u;
                const float dq = d0 * pw[q];
                Dq[q] = Aq[u].x;
                const bool valid = Aq[u].y >= 0.0f;                 // inside the frame (sink: R < 0)
                const bool in_r = fabsf(Aq[u].x + dq) <= Aq[u].y;
                const float sd = series_delta(make_float4(Aq[u].z, Aq[u].w, Bq[u].x, Bq[u].y), Aq[u].x, dq);
                fpart += in_r ? sd : 0.0f;
                fast |= in_r ? 1u << q : 0u;
                const bool dir = valid && !in_r;
                nevals += valid ? 1 : 0;
                ndirect += dir ? 1 : 0;
                const uint64_t bal = __ballot(dir);
                if (bal) {
                    const int slot = nq + lanes_below(bal);
                    const bool queued = dir && slot < WS_QCAP;
                    over |= (dir && !queued) ? 1u << q : 0u;
                    const int ws = queued ? slot : WS_QCAP;
                    jobs[ws] = make_float4(maq[u] + Aq[u].x, dq, pcq[q].x, pcq[q].y);
                    job_ri[ws] = ring_index(q);
                    nq += __popcll(bal);
                }
            }
        }
        // the commit reads the masks from these lane words (keeps the
        // compiler from holding one lane mask per entry in scalar registers)
        asm volatile("" : "+v"(fast), "+v"(over));
        // the next update's inputs (another pixel: its proposal does not
        // depend on this commit; the footprint records are per frame)
        if (nly < bh) prefetch(nly, nlx);
        wave_fence();
        // 2. the queued terms, one per lane, each keeping its window's
        //    recurrence state for the series at its new mean, formed after the
        //    decision if the move is accepted
        double part = (double)fpart;
        DirectKeep dk;
        dk.n4 = -1;
        float mu_j = 0.0f, d_j = 0.0f;
        int ri_j = NR;
        if (lane < min(nq, WS_QCAP)) {
            const float4 jb = jobs[lane];
            mu_j = jb.x;
            d_j = jb.y;
            ri_j = job_ri[lane];
            part += delta_ell_keep(mu_j, d_j, pc_from(jb.z, jb.w), nterms, dk);
        }
        // terms beyond the queue (rare): their owners, one entry at a time,
        // each rebuilt from the PSF order and the ring
        auto over_entry = [&](int q, int& ri, float& dq, int64_t& pix) {
            const int j = f.psf_order[lane + 64 * q];
            const int oy = j / s, ox = j - oy * s;
            int slot = ly % s + oy;
            slot = slot >= s ? slot - s : slot;
            ri = slot * RW + ox + lx;
            dq = d0 * f.psf[j];
            pix = m + (int64_t)(oy - r) * f.W + (ox - r);
        };
        if (nq > WS_QCAP) {
#pragma unroll 1
            for (int q = 0; q < NQ; ++q) {
                if ((over >> q) & 1) {
                    int ri;
                    float dq;
                    int64_t pix;
                    over_entry(q, ri, dq, pix);
                    part += delta_ell_notab(ring.ma[ri] + ring.A[ri].x, dq, load_pc(f.pc, pix), nterms);
                }
            }
        }
        part = wave_sum_dpp(part);
        // the decision (identical in every lane)
        const double delta = part + (double)hast;
        const bool acc = isfinite(delta) && ((double)logu < delta);
        if (lane == lx) {
            row_rho = acc ? rp : row_rho;
            row_acc = row_acc || acc;
            row_ls += gain * ((acc ? 1.0f : 0.0f) - 0.44f);
        }
        n_acc += acc ? 1 : 0;
        if (lane == 0) {
            if (dbg_delta) dbg_delta[base + m] = (float)delta;
            if (dbg_acc) dbg_acc[base + m] = acc ? 1 : 0;
        }
        if (acc) {
            // series entries move their displacement; the others write theirs
            // back unchanged (queued ones are re-anchored just after, in order)
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                ring.A[ring_index(q)].x = ((fast >> q) & 1) ? Dq[q] + d0 * pw[q] : Dq[q];
            // queued terms left their series' radius: re-anchor at the new mean
            const bool reanchor = ri_j != NR && d_j != 0.0f;
            const Series nx = series_kept(dk, mu_j, d_j);
            const int wr = reanchor ? ri_j : NR;
            ring.A[wr] = reanchor ? make_float4(0.0f, nx.R, nx.b.x, nx.b.y) : make_float4(0.0f, -1.0f, 0.0f, 0.0f);
            ring.B[wr] = make_float2(nx.b.z, nx.b.w);
            ring.ma[wr] = mu_j + d_j;
            nfused += reanchor ? 1 : 0;
            if (nq > WS_QCAP) {
#pragma unroll 1
                for (int q = 0; q < NQ; ++q) {
                    if ((over >> q) & 1) {
                        int ri;
                        float dq;
                        int64_t pix;
                        over_entry(q, ri, dq, pix);
                        if (dq != 0.0f) {
                            const float mu1 = (ring.ma[ri] + ring.A[ri].x) + dq;
                            const Series sr = series_at(mu1, load_pc(f.pc, pix), aterms);
                            ring.A[ri] = make_float4(0.0f, sr.R, sr.b.x, sr.b.y);
                            ring.B[ri] = make_float2(sr.b.z, sr.b.w);
                            ring.ma[ri] = mu1;
                            ++nanch;
                        }
                    }
                }
            }
        }
        wave_fence();                                               // commits before the next footprint reads
        ly = nly;
        lx = nlx;
    }
    row_end();
    if (lane == 0) atomicAdd(&S.accepts[chain], n_acc);
    series_store_rows<64>(f, S, base, ry0, rx0, RW, ly_cur, s, ring);
    count_work6(S.counters, nterms, nevals, ndirect, nanch, aterms, nfused);
}

template <int NQ>
__global__ void __launch_bounds__(64) k_wave_series(Frame f, State S, int burn_in, int B, int py, int px, int k0,
                                                    int k1, float* dbg_delta, uint8_t* dbg_acc, int nblk) {
    extern __shared__ double lds_d[];
    int bi, chain;
    if (!xcd_block(nblk, f.C, bi, chain)) return;
    wave_series_block<NQ>(f, S, burn_in, B, py, px, bi, chain, *S.t, k0, k1, dbg_delta, dbg_acc, lds_d);
}

// ---------------------------------------------------------------------------
// Moments after a sweep: Welford over post-burn-in sweeps, per-batch
// statistics (mean rho, mean and M2 of log rho) for R-hat and MCSE, and
// per-workgroup partials of the log-posterior at the current mu.
// ---------------------------------------------------------------------------
// One chunk of WG pixels of one chain.
template <bool EM>
__device__ void moments_chunk(const Frame& f, const State& S, const Prior& pr, const MomentBufs& M, int burn_in,
                              int chunk, int chain, int64_t t) {
    __shared__ double s_redm[WG / 64];
    const int64_t n = (int64_t)chunk * WG + threadIdx.x;
    double lp = 0.0;
    if (n < f.N) {
        const int64_t i = (int64_t)chain * f.N + n;
        const float x = S.rho[i];
        if (t >= burn_in) {
            const float k = (float)(t - burn_in + 1);
            const float mo = M.mean[i];
            const float dlt = x - mo;
            const float mn = mo + dlt / k;
            M.mean[i] = mn;
            M.m2[i] = (t == burn_in ? 0.0f : M.m2[i]) + dlt * (x - mn);
        }
        const int64_t b = t / M.rhat_block;
        if (b < M.max_batches) {
            const int64_t CN = (int64_t)f.C * f.N;
            float* bp = M.batch + b * 3 * CN + i;
            const float lx = logf(x);
            const int j = (int)(t - b * M.rhat_block);
            if (j == 0) {
                bp[0] = x; bp[CN] = lx; bp[2 * CN] = 0.0f;
            } else {
                const float kk = (float)(j + 1);
                bp[0] += (x - bp[0]) / kk;
                const float ml = bp[CN];
                const float dl = lx - ml;
                const float ml2 = ml + dl / kk;
                bp[CN] = ml2;
                bp[2 * CN] += dl * (lx - ml2);
            }
        }
        if (n < f.Np) lp = ell_abs_cam<EM>(f, S.mu[(int64_t)chain * f.Np + n], n);   // pixels: Np <= N
        if (pr.kind == 1) lp += (double)(pr.a - 1.0f) * log((double)x) - (double)pr.b * (double)x;
    }
    lp = wave_sum(lp);
    if ((threadIdx.x & 63) == 0) s_redm[threadIdx.x >> 6] = lp;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < WG / 64; ++w) tot += s_redm[w];
        M.lp_partial[(int64_t)chunk * f.C + chain] = tot;
    }
    __syncthreads();
}

template <bool EM>
__global__ void __launch_bounds__(WG) k_moments(Frame f, State S, Prior pr, MomentBufs M, int burn_in) {
    moments_chunk<EM>(f, S, pr, M, burn_in, blockIdx.x, blockIdx.y, *S.t);
}

// Fixed-order reduction of one chain's partials -> trace[t][chain].
__device__ void finalize_chain(int C, int nblk, const MomentBufs& M, int chain, int64_t t) {
    __shared__ double s_redf[WG];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += WG) v += M.lp_partial[(int64_t)b * C + chain];
    s_redf[threadIdx.x] = v;
    __syncthreads();
    for (int off = WG / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s_redf[threadIdx.x] += s_redf[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && t < M.max_sweeps) {
        double lp = s_redf[0];
        if (M.dir_part)
            for (int b = 0; b < M.n_chunks; ++b) lp += M.dir_part[(int64_t)b * C + chain];
        M.trace[t * C + chain] = lp;
    }
    __syncthreads();
}

// All chains' trace entries; then t += 1.
__global__ void __launch_bounds__(WG) k_finalize(int C, int nblk, MomentBufs M, int64_t* tp, int advance) {
    const int64_t t = *tp;
    for (int c = 0; c < C; ++c) finalize_chain(C, nblk, M, c, t);
    if (threadIdx.x == 0 && advance) *tp = t + 1;
}

template <bool EM>
__global__ void k_loglik(Frame f, const float* mu, double* out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= f.Np) return;
    out[n] = ell_abs_cam<EM>(f, mu[n], n);
}

// Split R-hat per pixel on log rho from batch statistics (Chan et al.'s
// pairwise combination of means and M2).  Sequences: each chain's batches
// [b_lo, b_lo + half) and [b_lo + half, b_lo + 2 half).
__global__ void k_rhat_map(Frame f, MomentBufs M, int b_lo, int half, float* rhat) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= f.N) return;
    const int64_t CN = (int64_t)f.C * f.N;
    const double nb = (double)M.rhat_block;
    const int m = 2 * f.C;
    double sum_mean = 0.0, sum_var = 0.0, sum_mean2 = 0.0;
    double L = 0.0;
    for (int c = 0; c < f.C; ++c)
        for (int h = 0; h < 2; ++h) {
            double cnt = 0.0, mean = 0.0, m2 = 0.0;
            for (int b = b_lo + h * half; b < b_lo + (h + 1) * half; ++b) {
                const float* bp = M.batch + (int64_t)b * 3 * CN + (int64_t)c * f.N + n;
                const double bm = (double)bp[CN], bq = (double)bp[2 * CN];
                const double tot = cnt + nb;
                const double dl = bm - mean;
                mean += dl * nb / tot;
                m2 += bq + dl * dl * cnt * nb / tot;
                cnt = tot;
            }
            L = cnt;
            const double var = m2 / (cnt - 1.0);
            sum_mean += mean;
            sum_mean2 += mean * mean;
            sum_var += var;
        }
    const double gm = sum_mean / m;
    const double Bv = L * (sum_mean2 - m * gm * gm) / (m - 1);
    const double Wv = sum_var / m;
    const double vplus = (L - 1.0) / L * Wv + Bv / L;
    rhat[n] = (float)sqrt(vplus / Wv);
}

// Histogram of R-hat values: n_fine bins of width w_fine from lo, then n_coarse
// bins of width w_coarse, then one overflow bin (NaN counts as overflow).
__global__ void k_hist(const float* v, int64_t n, float lo, float w_fine, int n_fine, float w_coarse, int n_coarse,
                       unsigned int* hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = v[i];
    int b;
    const float top_fine = lo + w_fine * n_fine;
    if (!(x == x)) b = n_fine + n_coarse;
    else if (x < top_fine) b = x < lo ? 0 : min((int)((x - lo) / w_fine), n_fine - 1);
    else b = n_fine + min((int)((x - top_fine) / w_coarse), n_coarse);
    atomicAdd(&hist[b], 1u);
}

// Batch-means MCSE of the posterior mean per pixel, pooled over chains.
__global__ void k_mcse(Frame f, MomentBufs M, int b0, int nb, float* out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= f.N) return;
    const int64_t CN = (int64_t)f.C * f.N;
    double acc = 0.0;
    for (int c = 0; c < f.C; ++c) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = b0; b < b0 + nb; ++b) {
            const double v = (double)M.batch[(int64_t)b * 3 * CN + (int64_t)c * f.N + n];
            s1 += v;
            s2 += v * v;
        }
        const double mean = s1 / nb;
        const double var = (s2 - nb * mean * mean) / (nb - 1);
        acc += fmax(var, 0.0) / nb;
    }
    out[n] = (float)sqrt(acc / ((double)f.C * f.C));
}

__global__ void k_pooled(Frame f, MomentBufs M, int64_t ns, int chain, float* mean, float* var) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= f.N) return;
    if (chain >= 0) {
        const int64_t i = (int64_t)chain * f.N + n;
        if (mean) mean[n] = M.mean[i];
        if (var) var[n] = M.m2[i] / (float)(ns - 1);
        return;
    }
    double m = 0.0;
    for (int c = 0; c < f.C; ++c) m += (double)M.mean[(int64_t)c * f.N + n];
    m /= f.C;
    double ss = 0.0;
    for (int c = 0; c < f.C; ++c) {
        const double dd = (double)M.mean[(int64_t)c * f.N + n] - m;
        ss += (double)M.m2[(int64_t)c * f.N + n] + (double)ns * dd * dd;
    }
    if (mean) mean[n] = (float)m;
    if (var) var[n] = (float)(ss / ((double)f.C * ns - 1.0));
}

__global__ void k_philox(const uint4* ctr, int64_t n, uint2 key, uint4* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], key);
}

__global__ void k_fill(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


// ---------------------------------------------------------------------------
// Learned part: the frame's photon scale, the network input, the learned warm
// start, and the block independence move.
// ---------------------------------------------------------------------------
// Per-workgroup partial sums of c = (w - o)/G -> part[wg] (double).
__global__ void k_sum_c(Frame f, double* part) {
    __shared__ double s_r[WG / 64];
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    double v = n < f.N ? (double)f.pc[n].x : 0.0;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) s_r[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < WG / 64; ++w) t += s_r[w];
        part[blockIdx.x] = t;
    }
}

// scale = mean c if that exceeds 1e-3 photons, else 1.  One workgroup.
__global__ void k_scale(const double* part, int nw, int64_t N, float* scale) {
    __shared__ double s_r[WG];
    double v = 0.0;
    for (int i = threadIdx.x; i < nw; i += WG) v += part[i];
    s_r[threadIdx.x] = v;
    __syncthreads();
    for (int off = WG / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s_r[threadIdx.x] += s_r[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = s_r[0] / (double)N;
        *scale = m > 1e-3 ? (float)m : 1.0f;
    }
}

// Network input on a zero-padded Hp x Wp grid: c / scale inside the frame.
__global__ void k_learned_input(Frame f, const float* scale, int Hp, int Wp, float* x) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= (int64_t)Hp * Wp) return;
    const int y = (int)(i / Wp), xx = (int)(i - (int64_t)y * Wp);
    x[i] = (y < f.H && xx < f.W) ? f.pc[(int64_t)y * f.W + xx].x / *scale : 0.0f;
}

// Proposal maps from the network output (m, s) and the warm start of every chain:
//   mean_log = m + log scale, sd_log = clamp(exp(s), 0.02, 3),
//   rho = exp(mean_log + sd_log xi), xi from the init stream at t = 0.
__global__ void k_learned_init(Frame f, State S, const float* out, int Wp, const float* scale, float log_step0,
                               float* pm, float* ps) {
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int chain = blockIdx.y;
    if (n >= f.N) return;
    const int y = (int)(n / f.W), x = (int)(n - (int64_t)y * f.W);
    const int64_t q = (int64_t)y * Wp + x;
    float m = out[2 * q] + logf(*scale);
    float sd = expf(out[2 * q + 1]);
    if (!isfinite(m)) m = logf(fmaxf(f.pc[n].x, 0.5f));
    sd = isfinite(sd) ? fminf(fmaxf(sd, 0.02f), 3.0f) : 1.0f;
    if (chain == 0) {
        pm[n] = m;
        ps[n] = sd;
    }
    // chains start overdispersed against the network's approximation (twice
    // its spread, at most 3 in log rho), as a between-chain R-hat requires
    const float xi = box_muller(draw(f.key, (uint32_t)n, 0u, (uint32_t)chain, STREAM_INIT));
    float v = expf(m + fminf(2.0f * sd, 3.0f) * xi);
    if (!(v > 0.0f) || !isfinite(v)) v = fmaxf(f.pc[n].x, 0.5f);
    const int64_t i = (int64_t)chain * f.N + n;
    S.rho[i] = v;
    S.log_step[i] = log_step0;
}

// One colour of the block independence move.  16 x 16 blocks; colour (cy, cx)
// of the period x period block colouring; one workgroup (one thread per block
// pixel) per (block, chain).  LDS: 1/k table, PSF, mu and d-mu of the
// (16 + 2r)^2 region.
constexpr int BS = 16;

template <bool EM>
__global__ void __launch_bounds__(WG) k_block_colour(Frame f, State S, Prior pr, const float* pm, const float* ps,
                                                     const double* inv_tab, int period, int cy, int cx,
                                                     uint32_t pass, float beta, float walk, unsigned long long* bacc,
                                                     float* dbg_delta, uint8_t* dbg_acc) {
    extern __shared__ double lds_b[];
    const int s = f.s, r = f.r, RW = BS + 2 * r;
    double* s_inv = lds_b;                              // [INV_TABLE]
    double* s_red = s_inv + INV_TABLE;                  // [WG / 64]
    float* s_psf = (float*)(s_red + WG / 64);           // [s*s]
    float* s_mu = s_psf + s * s;                        // [RW*RW], -1 outside the frame
    float* s_dmu = s_mu + RW * RW;                      // [RW*RW]
    float* s_d = s_dmu + RW * RW;                       // [BS*BS]
    __shared__ int s_flag;

    const int chain = blockIdx.y;
    const int nbx = (f.W + BS - 1) / BS;
    const int nbx_c = (nbx - cx + period - 1) / period;
    const int bi = blockIdx.x;
    const int by = cy + period * (bi / nbx_c), bx = cx + period * (bi % nbx_c);
    const int by0 = by * BS, bx0 = bx * BS;
    const int ry0 = by0 - r, rx0 = bx0 - r;
    const int64_t base = (int64_t)chain * f.N;

    for (int i = threadIdx.x; i < INV_TABLE; i += WG) s_inv[i] = inv_tab[i];
    for (int j = threadIdx.x; j < s * s; j += WG) s_psf[j] = f.psf[j];
    for (int i = threadIdx.x; i < RW * RW; i += WG) {
        const int yy = ry0 + i / RW, xx = rx0 + i % RW;
        s_mu[i] = (yy >= 0 && yy < f.H && xx >= 0 && xx < f.W) ? S.mu[base + (int64_t)yy * f.W + xx] : -1.0f;
    }
    // this thread's block pixel: proposal, log q(rho) - log q(rho'), prior ratio
    const int ty = threadIdx.x / BS, tx = threadIdx.x % BS;
    const int y = by0 + ty, x = bx0 + tx;
    double term = 0.0;
    float rp = 0.0f;
    float d = 0.0f;
    const bool inside = y < f.H && x < f.W;
    if (walk > 0.0f) {
        // Walk along what the blur removes: u' = u + walk h, h = xi - P (x)_B xi,
        // the blur of the block's white noise restricted to the block's pixels
        // in the frame; symmetric in u = log rho, so the log acceptance ratio
        // carries the Jacobian sum_m (u'_m - u_m).
        const int64_t m = (int64_t)y * f.W + x;
        const float xi = inside ? box_muller(draw(f.key, (uint32_t)m, pass, (uint32_t)chain, STREAM_BLOCK)) : 0.0f;
        s_d[threadIdx.x] = xi;
        __syncthreads();
        float h = 0.0f;
        if (inside) {
            float b = 0.0f;
            const int a0 = max(0, ty - r), a1 = min(BS - 1, ty + r);
            const int c0 = max(0, tx - r), c1 = min(BS - 1, tx + r);
            for (int a = a0; a <= a1; ++a) {
                const float* prow = s_psf + (ty - a + r) * s + (tx + r);
                const float* xrow = s_d + a * BS;
                for (int c = c0; c <= c1; ++c) b = fmaf(prow[-c], xrow[c], b);
            }
            h = xi - b;
        }
        __syncthreads();
        if (inside) {
            const float r0 = S.rho[base + m];
            const float hs = walk * h;
            rp = r0 * expf(hs);
            term = (double)hs;
            if (pr.kind == 1) term += (double)(pr.a - 1.0f) * (double)hs - (double)pr.b * ((double)rp - (double)r0);
            if (!(rp > 0.0f) || !isfinite(rp)) term = -INFINITY;
            d = rp - r0;
        }
    } else if (inside) {
        const int64_t m = (int64_t)y * f.W + x;
        const float r0 = S.rho[base + m];
        const float xi = box_muller(draw(f.key, (uint32_t)m, pass, (uint32_t)chain, STREAM_BLOCK));
        const float lm = pm[m], sd = ps[m];
        const float lr0 = logf(r0);
        const float z = (lr0 - lm) / sd;
        // autoregressive step around the reference N(lm, sd^2) in log rho;
        // beta = 1 draws independently of the current value
        const float zp = beta < 1.0f ? fmaf(sqrtf(1.0f - beta * beta), z, beta * xi) : xi;
        const float lrp = fmaf(sd, zp, lm);
        rp = expf(lrp);
        term = (double)(-lr0 - 0.5f * z * z) - (double)(-lrp - 0.5f * zp * zp);
        if (pr.kind == 1) term += (double)(pr.a - 1.0f) * ((double)lrp - (double)lr0) - (double)pr.b * ((double)rp - (double)r0);
        if (!(rp > 0.0f) || !isfinite(rp)) term = -INFINITY;
        d = rp - r0;
    }
    s_d[threadIdx.x] = d;
    __syncthreads();
    // d-mu over the region and the likelihood change
    int nterms = 0;
    double part = term;
    for (int j = threadIdx.x; j < RW * RW; j += WG) {
        const int ny = j / RW, nx = j % RW;
        float acc = 0.0f;
        const int t0 = max(0, ny - 2 * r), t1 = min(BS - 1, ny);
        const int u0 = max(0, nx - 2 * r), u1 = min(BS - 1, nx);
        for (int a = t0; a <= t1; ++a) {
            const float* prow = s_psf + (ny - a) * s + nx;
            const float* drow = s_d + a * BS;
            for (int b = u0; b <= u1; ++b) acc = fmaf(drow[b], prow[-b], acc);
        }
        s_dmu[j] = acc;
        const float muv = s_mu[j];
        if (muv < 0.0f || acc == 0.0f) continue;
        const int64_t n = (int64_t)(ry0 + ny) * f.W + (rx0 + nx);
        part += delta_pix<EM>(muv, acc, load_pc(f.pc, n), s_inv, nterms);
    }
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < WG / 64; ++w) tot += s_red[w];
        const int64_t m0 = (int64_t)by0 * f.W + bx0;
        const float logu = logf(u01(draw(f.key, (uint32_t)m0, pass, (uint32_t)chain, STREAM_BLOCK_ACCEPT).x));
        const bool acc = isfinite(tot) && ((double)logu < tot);
        s_flag = acc ? 1 : 0;
        if (acc) atomicAdd(bacc, 1ull);
        const int64_t nblk = (int64_t)gridDim.x;
        if (dbg_delta) dbg_delta[(int64_t)chain * nblk + bi] = (float)tot;
        if (dbg_acc) dbg_acc[(int64_t)chain * nblk + bi] = acc ? 1 : 0;
    }
    __syncthreads();
    if (!s_flag) return;
    if (y < f.H && x < f.W) S.rho[base + (int64_t)y * f.W + x] = rp;
    for (int j = threadIdx.x; j < RW * RW; j += WG) {
        if (s_mu[j] < 0.0f) continue;
        const int yy = ry0 + j / RW, xx = rx0 + j % RW;
        S.mu[base + (int64_t)yy * f.W + xx] = s_mu[j] + s_dmu[j];
    }
}

// Training pair of one frame: the network input x = c / scale and the targets
// (mean of log(rho/scale), log std of log rho) of the log-normal with the
// posterior's mean and variance of rho.
__global__ void k_training_targets(Frame f, const float* mean, const float* var, const float* scale, float* x,
                                   float* tgt) {
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (n >= f.N) return;
    const float sc = *scale;
    x[n] = f.pc[n].x / sc;
    const float m = fmaxf(mean[n], 1e-12f);
    const float s2 = log1pf(fmaxf(var[n], 0.0f) / (m * m));
    tgt[2 * n] = logf(m / sc) - 0.5f * s2;
    tgt[2 * n + 1] = 0.5f * logf(fmaxf(s2, 1e-8f));
}

// Mean of rho over batches [b0, b0 + nb) of every chain (the R-hat window).
__global__ void k_window_mean(Frame f, MomentBufs M, int b0, int nb, float* out) {
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (n >= f.N) return;
    const int64_t CN = (int64_t)f.C * f.N;
    double s = 0.0;
    for (int c = 0; c < f.C; ++c)
        for (int b = b0; b < b0 + nb; ++b) s += (double)M.batch[(int64_t)b * 3 * CN + (int64_t)c * f.N + n];
    out[n] = (float)(s / ((double)f.C * nb));
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_pixel_consts(const Frame& f, float4* pc, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_pixel_consts, dim3(grid1(f.Np)), dim3(WG), 0, st, f, pc, bad);
    return hipGetLastError();
}

hipError_t launch_init_state(const Frame& f, const State& S, const float* rho0, float log_step0, int* bad,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_init_state, dim3(grid1(f.N), f.C), dim3(WG), 0, st, f, S, rho0, log_step0, bad);
    return hipGetLastError();
}

hipError_t launch_forward_propose(const Frame& f, const State& S, const Prior& pr, int propose, hipStream_t st) {
    if (f.sub > 1) {
        hipLaunchKernelGGL(k_forward_sub, dim3(grid1(f.Np), f.C), dim3(WG), 0, st, f, S);
        if (propose) hipLaunchKernelGGL(k_propose_sub, dim3(grid1(f.N), f.C), dim3(WG), 0, st, f, S, pr);
        return hipGetLastError();
    }
    const int nt = ((f.H + FT - 1) / FT) * ((f.W + FT - 1) / FT);
    hipLaunchKernelGGL(k_forward_propose, dim3(nt, f.C), dim3(WG), forward_lds(f.s), st, f, S, pr, propose);
    return hipGetLastError();
}

hipError_t launch_colour_pass(const Frame& f, const State& S, int burn_in, const double* inv_tab, int colour,
                              float* dbg_delta, uint8_t* dbg_acc, hipStream_t st) {
    if (f.sub > 1) {
        // colours: phase-major, then the pixel position mod s
        const int phase = colour / (f.s * f.s), cy = (colour % (f.s * f.s)) / f.s, cx = colour % f.s;
        if (phase >= f.sub * f.sub) return hipErrorInvalidValue;
        if (cy >= f.Hp || cx >= f.Wp) return hipSuccess;
        const int nrow = (f.Hp - cy + f.s - 1) / f.s, ncol = (f.Wp - cx + f.s - 1) / f.s;
        hipLaunchKernelGGL(f.camera ? k_colour_pass_sub<true> : k_colour_pass_sub<false>, dim3(nrow * ncol, f.C),
                           dim3(WG), 0, st, f, S, burn_in, inv_tab, phase, cy, cx, dbg_delta, dbg_acc);
        return hipGetLastError();
    }
    const int cy = colour / f.s, cx = colour % f.s;
    if (cy >= f.H || cx >= f.W) return hipSuccess;
    const int nrow = (f.H - cy + f.s - 1) / f.s, ncol = (f.W - cx + f.s - 1) / f.s;
    hipLaunchKernelGGL(f.camera ? k_colour_pass<true> : k_colour_pass<false>, dim3(nrow * ncol, f.C), dim3(WG), 0,
                       st, f, S, burn_in, inv_tab, cy, cx, dbg_delta, dbg_acc);
    return hipGetLastError();
}

size_t block_phase_lds(int B, int s) {
    const int RW = B + 2 * (s / 2);
    return (size_t)(INV_TABLE + MAX_ACT * (WG / 64)) * sizeof(double) + (size_t)(s * s + RW * RW) * sizeof(float) +
           (size_t)(s * s) * sizeof(uint16_t) + (size_t)RW * RW;
}

size_t block_phase_sub_lds(int B, int s, int k) {
    const int RW = B + 2 * (s / 2);
    return (size_t)(INV_TABLE + MAX_ACT * WAVES) * sizeof(double) + (size_t)(k * k * s * s + RW * RW) * sizeof(float) +
           (size_t)(s * s) * sizeof(uint16_t);
}

// Grid of a block scan over nblk blocks and C chains (xcd_block): ids
// 0 .. XCDS * C * ceil(nblk / XCDS) - 1 in dispatch order (x fastest), rows of
// up to 65536 groups of XCDS * C workgroups.
static dim3 xcd_grid(int nblk, int C) {
    const int nq = (nblk + XCDS - 1) / XCDS;
    const int qx = std::min(nq, 65536);
    return dim3((unsigned)(XCDS * C * qx), (unsigned)((nq + qx - 1) / qx));
}

hipError_t launch_block_phase(const Frame& f, const State& S, int burn_in, const double* inv_tab, int B,
                              int phase, int k0, int k1, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st) {
    if (f.sub > 1) {
        const int py = phase / 2, px = phase % 2;
        const int nby = (f.Hp + B - 1) / B, nbx = (f.Wp + B - 1) / B;
        const int nby_p = (nby - py + 1) / 2, nbx_p = (nbx - px + 1) / 2;
        if (nby_p <= 0 || nbx_p <= 0) return hipSuccess;
        const size_t lds = block_phase_sub_lds(B, f.s, f.sub);
        if (B < f.s - 1 || B < 1 || B > 4 * f.s || lds > 64 * 1024 || f.dir_am1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(f.camera ? k_block_phase_sub<true> : k_block_phase_sub<false>,
                           xcd_grid(nby_p * nbx_p, f.C), dim3(WG), lds, st, f, S, burn_in, inv_tab, B, py, px, k0, k1,
                           dbg_delta, dbg_acc, nby_p * nbx_p);
        return hipGetLastError();
    }
    const int py = phase / 2, px = phase % 2;
    const int nby = (f.H + B - 1) / B, nbx = (f.W + B - 1) / B;
    const int nby_p = (nby - py + 1) / 2, nbx_p = (nbx - px + 1) / 2;
    if (nby_p <= 0 || nbx_p <= 0) return hipSuccess;
    if (f.dir_am1) {
        // the chunk prior couples a block's pixels: one pixel per block and colour
        if (B != f.dir_B || B > f.s || B > DIR_MAX_B || f.s * f.s > SORT_MAX_F) return hipErrorInvalidValue;
        const size_t lds = block_phase_lds(B, f.s) + dir_lds_bytes(B);
        auto kern = f.camera ? k_block_phase_dir<true> : k_block_phase_dir<false>;
        static bool attr_set[2] = {false, false};
        if (!attr_set[f.camera ? 1 : 0]) {
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               80 * 1024);
            if (e != hipSuccess) return e;
            attr_set[f.camera ? 1 : 0] = true;
        }
        hipLaunchKernelGGL(kern, xcd_grid(nby_p * nbx_p, f.C), dim3(WG), lds, st, f, S, burn_in, inv_tab,
                           B, py, px, k0, k1, dbg_delta, dbg_acc, nby_p * nbx_p);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(f.camera ? k_block_phase<true> : k_block_phase<false>, xcd_grid(nby_p * nbx_p, f.C),
                       dim3(WG), block_phase_lds(B, f.s), st, f, S, burn_in, inv_tab, B, py, px, k0, k1, dbg_delta,
                       dbg_acc, nby_p * nbx_p);
    return hipGetLastError();
}

int chunk_count(const Frame& f) {
    const int B = f.dir_B;
    return B > 0 ? ((f.H + B - 1) / B) * ((f.W + B - 1) / B) : 0;
}

static size_t chunk_fourier_lds(int B) { return (size_t)(3 * B * B + 4 * B + WAVES) * sizeof(double); }

hipError_t launch_chunk_spectra(const Frame& f, const State& S, hipStream_t st) {
    if (!f.dir_am1) return hipSuccess;
    MomentBufs M{};
    hipLaunchKernelGGL(k_chunk_fourier<0>, dim3(chunk_count(f), f.C), dim3(WG), chunk_fourier_lds(f.dir_B), st, f,
                       S, M);
    return hipGetLastError();
}

hipError_t launch_chunk_logprior(const Frame& f, const State& S, const MomentBufs& M, hipStream_t st) {
    if (!f.dir_am1 || !M.dir_part) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_fourier<1>, dim3(chunk_count(f), f.C), dim3(WG), chunk_fourier_lds(f.dir_B), st, f,
                       S, M);
    return hipGetLastError();
}

size_t block_series_lds(int B, int s) {
    const int RW = B + 2 * (s / 2);
    return (size_t)2 * (WG / 64) * sizeof(double) + (size_t)s * RW * (sizeof(float4) + sizeof(float2) + sizeof(float));
}

bool block_series_fits(int B, int s) {
    return B <= s && B >= s - 1 && B >= 1 && s * s <= SER_Q * WG && block_series_lds(B, s) <= BLOCK_SERIES_LDS_MAX;
}

size_t wave_series_lds(int B, int s) {
    const int RW = B + 2 * (s / 2);
    return (WS_QCAP + 1) * (sizeof(float4) + sizeof(int)) +
           ((size_t)s * RW + 1) * (sizeof(float4) + sizeof(float2) + sizeof(float));
}

bool wave_series_fits(int B, int s) {
    return B <= s && 2 * B >= s - 1 && B >= 1 && s * s <= WS_NQ * 64 && wave_series_lds(B, s) <= 64 * 1024;
}

hipError_t launch_wave_series(const Frame& f, const State& S, int burn_in, int B, int phase, int k0, int k1,
                              float* dbg_delta, uint8_t* dbg_acc, hipStream_t st) {
    if (!wave_series_fits(B, f.s)) return hipErrorInvalidValue;
    const int py = phase / 3, px = phase % 3;
    const int nby = (f.H + B - 1) / B, nbx = (f.W + B - 1) / B;
    const int nby_p = (nby - py + 2) / 3, nbx_p = (nbx - px + 2) / 3;
    if (nby_p <= 0 || nbx_p <= 0) return hipSuccess;
    const size_t lds = wave_series_lds(B, f.s);
    const int F = f.s * f.s;
    const dim3 grid = xcd_grid(nby_p * nbx_p, f.C);
    if (F <= 4 * 64)
        hipLaunchKernelGGL(k_wave_series<4>, grid, dim3(64), lds, st, f, S, burn_in, B, py, px, k0, k1, dbg_delta,
                           dbg_acc, nby_p * nbx_p);
    else if (F <= 8 * 64)
        hipLaunchKernelGGL(k_wave_series<8>, grid, dim3(64), lds, st, f, S, burn_in, B, py, px, k0, k1, dbg_delta,
                           dbg_acc, nby_p * nbx_p);
    else
        hipLaunchKernelGGL(k_wave_series<16>, grid, dim3(64), lds, st, f, S, burn_in, B, py, px, k0, k1, dbg_delta,
                           dbg_acc, nby_p * nbx_p);
    return hipGetLastError();
}

hipError_t launch_block_series(const Frame& f, const State& S, int burn_in, const double* inv_tab, int B, int phase,
                               int k0, int k1, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st) {
    if (!block_series_fits(B, f.s)) return hipErrorInvalidValue;
    const int py = phase / 2, px = phase % 2;
    const int nby = (f.H + B - 1) / B, nbx = (f.W + B - 1) / B;
    const int nby_p = (nby - py + 1) / 2, nbx_p = (nbx - px + 1) / 2;
    if (nby_p <= 0 || nbx_p <= 0) return hipSuccess;
    const size_t lds = block_series_lds(B, f.s);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_block_series, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)BLOCK_SERIES_LDS_MAX);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    (void)inv_tab;   // the pass computes its reciprocals (no table in its LDS budget)
    const int nblk = nby_p * nbx_p;
    hipLaunchKernelGGL(k_block_series, xcd_grid(nblk, f.C), dim3(WG), lds, st, f, S, burn_in, B, py, px, k0, k1,
                       dbg_delta, dbg_acc, nblk);
    return hipGetLastError();
}

hipError_t launch_moments(const Frame& f, const State& S, const Prior& pr, const MomentBufs& M, int burn_in,
                          int advance, hipStream_t st) {
    const unsigned nblk = grid1(f.N);
    hipLaunchKernelGGL(f.camera ? k_moments<true> : k_moments<false>, dim3(nblk, f.C), dim3(WG), 0, st, f, S, pr, M,
                       burn_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_chunk_logprior(f, S, M, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, st, f.C, (int)nblk, M, S.t, advance);
    return hipGetLastError();
}

hipError_t launch_loglik(const Frame& f, const float* mu, double* out, hipStream_t st) {
    hipLaunchKernelGGL(f.camera ? k_loglik<true> : k_loglik<false>, dim3(grid1(f.Np)), dim3(WG), 0, st, f, mu, out);
    return hipGetLastError();
}

hipError_t launch_rhat_map(const Frame& f, const MomentBufs& M, int b_lo, int half, float* rhat, hipStream_t st) {
    hipLaunchKernelGGL(k_rhat_map, dim3(grid1(f.N)), dim3(WG), 0, st, f, M, b_lo, half, rhat);
    return hipGetLastError();
}

hipError_t launch_hist(const float* v, int64_t n, float lo, float w_fine, int n_fine, float w_coarse, int n_coarse,
                       unsigned int* hist, hipStream_t st) {
    hipLaunchKernelGGL(k_hist, dim3(grid1(n)), dim3(WG), 0, st, v, n, lo, w_fine, n_fine, w_coarse, n_coarse, hist);
    return hipGetLastError();
}

hipError_t launch_mcse(const Frame& f, const MomentBufs& M, int b0, int nb, float* mcse, hipStream_t st) {
    hipLaunchKernelGGL(k_mcse, dim3(grid1(f.N)), dim3(WG), 0, st, f, M, b0, nb, mcse);
    return hipGetLastError();
}

hipError_t launch_pooled_moments(const Frame& f, const MomentBufs& M, int64_t n, int chain, float* mean,
                                 float* var, hipStream_t st) {
    hipLaunchKernelGGL(k_pooled, dim3(grid1(f.N)), dim3(WG), 0, st, f, M, n, chain, mean, var);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, int64_t n, uint2 key, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_philox, dim3(grid1(n)), dim3(WG), 0, st, (const uint4*)ctr, n, key, (uint4*)out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(WG), 0, st, p, n, v);
    return hipGetLastError();
}

int block_period(int r) { return 1 + (2 * r + BS - 1) / BS; }

int block_colour_count(const Frame& f, int colour) {
    const int P = block_period(f.r);
    const int cy = colour / P, cx = colour % P;
    const int nby = (f.H + BS - 1) / BS, nbx = (f.W + BS - 1) / BS;
    if (cy >= nby || cx >= nbx) return 0;
    return ((nby - cy + P - 1) / P) * ((nbx - cx + P - 1) / P);
}

size_t block_colour_lds(int s) {
    const int RW = BS + s - 1;
    return (size_t)(INV_TABLE + WG / 64) * sizeof(double) + (size_t)(s * s + 2 * RW * RW + BS * BS) * sizeof(float);
}

hipError_t launch_block_colour(const Frame& f, const State& S, const Prior& pr, const float* pm, const float* ps,
                               const double* inv_tab, int colour, uint32_t pass, float beta, float walk,
                               unsigned long long* bacc, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st) {
    const int P = block_period(f.r);
    const int nb = block_colour_count(f, colour);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(f.camera ? k_block_colour<true> : k_block_colour<false>, dim3(nb, f.C), dim3(WG),
                       block_colour_lds(f.s), st, f, S, pr, pm, ps, inv_tab, P, colour / P, colour % P, pass, beta,
                       walk, bacc, dbg_delta, dbg_acc);
    return hipGetLastError();
}

hipError_t launch_training_targets(const Frame& f, const float* mean, const float* var, const float* scale, float* x,
                                   float* tgt, hipStream_t st) {
    hipLaunchKernelGGL(k_training_targets, dim3(grid1(f.N)), dim3(WG), 0, st, f, mean, var, scale, x, tgt);
    return hipGetLastError();
}

hipError_t launch_window_mean(const Frame& f, const MomentBufs& M, int b0, int nb, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_window_mean, dim3(grid1(f.N)), dim3(WG), 0, st, f, M, b0, nb, out);
    return hipGetLastError();
}

hipError_t launch_frame_scale(const Frame& f, double* part, float* scale, hipStream_t st) {
    const unsigned nw = grid1(f.N);
    hipLaunchKernelGGL(k_sum_c, dim3(nw), dim3(WG), 0, st, f, part);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(WG), 0, st, part, (int)nw, f.N, scale);
    return hipGetLastError();
}

hipError_t launch_learned_input(const Frame& f, const float* scale, int Hp, int Wp, float* x, hipStream_t st) {
    hipLaunchKernelGGL(k_learned_input, dim3(grid1((int64_t)Hp * Wp)), dim3(WG), 0, st, f, scale, Hp, Wp, x);
    return hipGetLastError();
}

hipError_t launch_learned_init(const Frame& f, const State& S, const float* out, int Wp, const float* scale,
                               float log_step0, float* pm, float* ps, hipStream_t st) {
    hipLaunchKernelGGL(k_learned_init, dim3(grid1(f.N), f.C), dim3(WG), 0, st, f, S, out, Wp, scale, log_step0, pm,
                       ps);
    return hipGetLastError();
}

}  // namespace bdc

namespace bdc {
namespace {

__global__ void k_batch_advance(int64_t* const* tps, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *tps[i] += 1;
}

// One item per workgroup: every item of one segment (one level, one kind of
// work, all tiles and chains).  Items of a segment are independent; the
// segment before finished with the previous launch, so no workgroup ever
// waits for another.
// Three waves per SIMD, as for the single-frame block-series kernel: the
// tile descriptor's indirection would otherwise take the series body just past
// the register count at which three fit.
template <int KIND>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3)))
k_batch(const TileDesc* tiles, const Item* items, const double* inv_tab) {
    extern __shared__ double lds_b[];
    const Item I = items[blockIdx.x];
    const TileDesc& T = tiles[I.tile];
    const int64_t t = *T.S.t;
    const int ph = I.level - 1;
    if constexpr (KIND == BK_FORWARD) {
        forward_tile(T.f, T.S, T.pr, 1, I.index, I.chain, t, (float*)lds_b);
    } else if constexpr (KIND == BK_SERIES) {
        block_series_block(T.f, T.S, T.burn_in, T.B, ph / 2, ph % 2, I.index, I.chain, t, 0, T.f.s * T.f.s,
                           nullptr, nullptr, lds_b);
    } else if constexpr (KIND == BK_PHASE || KIND == BK_PHASE_EM) {
        block_phase_block<false, KIND == BK_PHASE_EM>(T.f, T.S, T.burn_in, inv_tab, T.B, ph / 2, ph % 2, I.index,
                                                      I.chain, t, 0, T.f.s * T.f.s, nullptr, nullptr, lds_b);
    } else if constexpr (KIND == BK_MOMENTS || KIND == BK_MOMENTS_EM) {
        moments_chunk<KIND == BK_MOMENTS_EM>(T.f, T.S, T.pr, T.M, T.burn_in, I.index, I.chain, t);
    } else {
        finalize_chain(T.f.C, T.count[LEV_MOMENTS], T.M, I.chain, t);
    }
}

// Nine-phase block-series items: one wavefront each.
template <int NQ>
__global__ void __launch_bounds__(64) k_batch_wave(const TileDesc* tiles, const Item* items) {
    extern __shared__ double lds_b[];
    const Item I = items[blockIdx.x];
    const TileDesc& T = tiles[I.tile];
    const int ph = I.level - 1;
    wave_series_block<NQ>(T.f, T.S, T.burn_in, T.B, ph / 3, ph % 3, I.index, I.chain, *T.S.t, 0, T.f.s * T.f.s,
                          nullptr, nullptr, lds_b);
}

}  // namespace

size_t forward_lds(int s) {
    const int TWd = FT + 2 * (s / 2);
    return (size_t)(TWd * TWd + s * s) * sizeof(float);
}

hipError_t launch_batch_level(int kind, const TileDesc* tiles, const Item* items, int n_items,
                              const double* inv_tab, size_t lds, hipStream_t st) {
    if (n_items <= 0) return hipSuccess;
    const dim3 g(n_items), blk(WG);
    switch (kind) {
        case BK_FORWARD: hipLaunchKernelGGL(k_batch<BK_FORWARD>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_SERIES: hipLaunchKernelGGL(k_batch<BK_SERIES>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_PHASE: hipLaunchKernelGGL(k_batch<BK_PHASE>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_MOMENTS: hipLaunchKernelGGL(k_batch<BK_MOMENTS>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_FINALIZE: hipLaunchKernelGGL(k_batch<BK_FINALIZE>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_WAVE4: hipLaunchKernelGGL(k_batch_wave<4>, g, dim3(64), lds, st, tiles, items); break;
        case BK_WAVE8: hipLaunchKernelGGL(k_batch_wave<8>, g, dim3(64), lds, st, tiles, items); break;
        case BK_WAVE16: hipLaunchKernelGGL(k_batch_wave<16>, g, dim3(64), lds, st, tiles, items); break;
        case BK_PHASE_EM: hipLaunchKernelGGL(k_batch<BK_PHASE_EM>, g, blk, lds, st, tiles, items, inv_tab); break;
        case BK_MOMENTS_EM:
            hipLaunchKernelGGL(k_batch<BK_MOMENTS_EM>, g, blk, lds, st, tiles, items, inv_tab);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_advance(int64_t* const* tps, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_advance, dim3((n + WG - 1) / WG), dim3(WG), 0, st, tps, n);
    return hipGetLastError();
}

}  // namespace bdc
