// bdc_device.h -- device arithmetic of the gfx950 sampler: counter-based random
// numbers and the per-pixel likelihood of the paper's camera model.
//
// Pixel model (Methods, Eqs. 3-6):  with c = (w - o)/G and a = G^2/(2 sigma^2),
//   L(mu) = (2 pi sigma^2)^-1/2 * sum_{k>=0} exp(-a (k - c)^2) mu^k e^-mu / k!.
// Summands are log-concave in k.  Their ratio r_k = W_{k+1}/W_k =
// mu exp(-a (2k + 1 - 2c)) / (k + 1) is a geometric sequence in exp(2a) times
// 1/(k+1), which is what the inner loops below iterate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdc_consts.h"

namespace bdc {

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// Ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint4 philox4x32_10(uint4 ctr, uint2 key) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * ctr.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * ctr.z;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        ctr = make_uint4(h1 ^ ctr.y ^ key.x, l1, h0 ^ ctr.w ^ key.y, l0);
        key.x += 0x9E3779B9u;
        key.y += 0xBB67AE85u;
    }
    return ctr;
}

// Random-number streams of one (pixel, sweep, chain) counter.
enum : uint32_t { STREAM_PROPOSAL = 0, STREAM_ACCEPT = 1, STREAM_INIT = 2, STREAM_BLOCK = 3, STREAM_BLOCK_ACCEPT = 4 };

__device__ inline uint4 draw(uint2 key, uint32_t pixel, uint32_t sweep, uint32_t chain, uint32_t stream) {
    return philox4x32_10(make_uint4(pixel, sweep, chain, stream), key);
}

// Open-interval uniform from the top 23 bits: ((x >> 9) + 1/2) 2^-23, exact in FP32.
__device__ inline float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

// Box-Muller from words 0 and 1 of one block (cosine branch).
__device__ inline float box_muller(uint4 r) {
    const float u1 = u01(r.x), u2 = u01(r.y);
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// ---------------------------------------------------------------------------
// Constants of the phi window and the ratio recurrence.
// ---------------------------------------------------------------------------
// Above this a the geometric factor exp(2a) leaves FP32 range: those pixels
// (read noise far below one photon) take a short direct-exponent loop.
constexpr float A_RECUR_MAX = 40.0f;
// Depth of the phi window: every omitted summand is below the largest by
// exp(-TAIL_T) at least (log-concavity bound), total < 1e-8 relative.
constexpr float TAIL_T = 20.0f;

// Per-pixel constants of one footprint evaluation.  Stored per pixel (one
// 16-byte record, derived once per frame): c, 2a, and L0 = 2a(c - ks) -
// log(ks + 1), iB = 1/(2a + 1/(ks + 1)) with ks = max(c, 0), so that the
// tangent step of L (below) at ks is ks + (L0 + log mu) iB.  Derived in
// registers at load: ks, 1/(2a) and h0 = sqrt(TAIL_T / a), the half-width
// bound from the curvature 2a.  (16 bytes keep a workgroup's footprint of
// records small enough for the resident workgroups of an XCD to share its L2.)
struct PixConst {
    float c, a2, inv2a;
    float ks, L0, iB, h0;
};

__device__ inline float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ inline float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// log(1 + x) to a few ulp.  |x| < 1/16: the Taylor series through x^8
// (remainder below x^9/9, < 3e-11 relative).  Otherwise the hardware log of
// u = fl(1 + x) with Kahan's correction log1p(x) = log(u) x / (u - 1), which
// cancels the rounding of u; there |log u| > 0.06, where the hardware log's
// error is a few ulp of the result.
__device__ inline float log1p_k(float x) {
    float s = fmaf(x, -0.125f, 0.14285714285714285f);
    s = fmaf(x, s, -0.16666666666666666f);
    s = fmaf(x, s, 0.2f);
    s = fmaf(x, s, -0.25f);
    s = fmaf(x, s, 0.33333333333333333f);
    s = fmaf(x, s, -0.5f);
    s = fmaf(x, s, 1.0f);
    const float series = x * s;
    const float u = 1.0f + x;
    const float kahan = fast_ln(u) * (x * fast_rcp(u - 1.0f));
    return fabsf(x) < 0.0625f ? series : kahan;
}

// exp(y) in double with FP32 relative accuracy over the whole double range:
// 2^(y log2 e) = 2^n * 2^f, f in [0, 1) through the FP32 exp2.
__device__ inline double exp_wide(double y) {
    const double z = y * 1.4426950408889634;
    const double n = floor(z);
    const float f = (float)(z - n);
    return ldexp((double)__builtin_amdgcn_exp2f(f), (int)fmax(fmin(n, 2000.0), -2000.0));
}

// The same for |y| < 2^30 (no clamp of the exponent; ldexp saturates).
__device__ inline double exp_wide_b(double y) {
    const double z = y * 1.4426950408889634;
    const double n = floor(z);
    const float f = (float)(z - n);
    return ldexp((double)__builtin_amdgcn_exp2f(f), (int)n);
}

// exp(y) for 0 < y <= 2 A_RECUR_MAX in FP32 range, FP32 relative accuracy.
__device__ inline double exp_small(float y) {
    const double z = (double)y * 1.4426950408889634;
    const double n = floor(z);
    const float f = (float)(z - n);
    return (double)__builtin_amdgcn_ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
}

// 1/n, 1/(n-1), 1/(n-2), 1/(n-3) for 4 <= n < 2^20 from one hardware
// reciprocal of their product and one Newton step: each reciprocal is the
// product of the other three factors with it (relative error below 1e-15).
__device__ inline void recip4(int n, double cv[4]) {
    const double na = (double)n, nb = na - 1.0, nc = na - 2.0, nd = na - 3.0;
    const double pab = na * nb, pcd = nc * nd, P = pab * pcd;
    double R = __builtin_amdgcn_rcp(P);
    R = fma(R, fma(-P, R, 1.0), R);
    const double Rab = R * pab, Rcd = R * pcd;
    cv[0] = nb * Rcd;
    cv[1] = na * Rcd;
    cv[2] = nd * Rab;
    cv[3] = nc * Rab;
}

// ---------------------------------------------------------------------------
// phi window.  For mean mu the log-summand f(k) = -a (k-c)^2 + k log mu - lgamma(k+1)
// is concave with f'' <= -(2a + 1/(k+1)).  Its continuous mode k* lies where
//   2a(c - k) + log mu - digamma(k + 1) = 0,  and log(k+1/2) < digamma(k+1) < log(k+1).
// Lower bound: L(k) = 2a(c - k) + log mu - log(k + 1) is convex and decreasing
// with L(k*) >= 0, so one tangent (Newton) step from any point lands at or below
// its root, hence below k*.  Upper bound: for k >= p, log(k + 1/2) >= log(p + 1/2)
// so f'(k) < 2a(c - k) + log mu - log(p + 1/2) <= 0 once k >= c + log(mu/(p+1/2))/(2a).
// The window is [p - h, q + h] with h^2 = 2 TAIL_T / kappa, kappa a lower bound on
// the curvature: 2a, and 1/(2q + 4T + 2) (h <= q + 4T + 1).  mu enters
// monotonically, so the window of [mu_lo, mu_hi] covers both the current and
// the proposed mean.
// ---------------------------------------------------------------------------
struct Window { int lo, hi; bool ok; };

__device__ inline Window finish_window(float p, float q, float h0) {
    // hardware square root: the half-width only needs a few significant digits
    const float hp = __builtin_amdgcn_sqrtf(2.0f * TAIL_T * (2.0f * q + 4.0f * TAIL_T + 2.0f));
    const float h = fminf(h0, hp);
    Window w;
    // photon counts beyond 2^20 per pixel are outside the model's working range
    // (and would make the loops unbounded): flagged, the caller rejects
    w.ok = (q + h < 1048576.0f);
    w.lo = w.ok ? (int)fmaxf(floorf(p - h), 0.0f) : 0;
    w.hi = w.ok ? (int)ceilf(q + h) : 0;
    return w;
}

// Newton refinement of the lower bound (slow path for a loose bracket); the
// bracket travels in registers (by value), so the common path touches no
// private memory.
__device__ __noinline__ float2 refine_bracket(float lmu_lo, float lmu_hi, PixConst pc, float2 pq) {
    float p = pq.x, q = pq.y;
    for (int it = 0; it < 8 && q - p > 6.0f; ++it) {
        const float k1 = p + 1.0f;
        const float L = pc.a2 * (pc.c - p) + lmu_lo - fast_ln(k1);
        const float pn = fmaxf(fmaf(L * k1, fast_rcp(fmaf(pc.a2, k1, 1.0f)), p), 0.0f);
        if (pn - p < 0.25f) break;
        p = pn;
        q = fmaxf(p, pc.c + (lmu_hi - fast_ln(p + 0.5f)) * pc.inv2a);
    }
    return make_float2(p, q);
}

__device__ inline Window phi_window(float lmu_lo, float lmu_hi, const PixConst& pc) {
    float2 pq;
    pq.x = fmaxf(fmaf(pc.L0 + lmu_lo, pc.iB, pc.ks), 0.0f);
    pq.y = fmaxf(pq.x, pc.c + (lmu_hi - fast_ln(pq.x + 0.5f)) * pc.inv2a);
    if (pq.y - pq.x > 6.0f) pq = refine_bracket(lmu_lo, lmu_hi, pc, pq);
    return finish_window(pq.x, pq.y, pc.h0);
}

// log(num / den) for positive double sums, to FP32 relative accuracy of the
// result at every scale, in one branch-free path: the ratio's binary exponent
// is split off in double with the mantissa m scaled into [sqrt(1/2), sqrt(2)),
// and log m = 2 atanh(z), z = (m - 1)/(m + 1), |z| <= 0.1716, by its odd
// series through z^9 (remainder below 5e-9 relative).  m - 1 is exact in
// double, so ratios near 1 keep their small logarithm to full relative
// accuracy, and ratios far from 1 (a proposal far from the current state)
// never round against 1.
__device__ inline double log_ratio(double num, double den) {
    const double q = num * __builtin_amdgcn_rcp(den);
    int e = __builtin_amdgcn_frexp_exp(q);
    double m = __builtin_amdgcn_frexp_mant(q);           // [1/2, 1)
    if (m < 0.70710678118654752) { m += m; e -= 1; }     // [sqrt(1/2), sqrt(2))
    const float z = (float)((m - 1.0) * __builtin_amdgcn_rcp(m + 1.0));
    const float z2 = z * z;
    float poly = fmaf(z2, 0.22222222222222222f, 0.28571428571428571f);
    poly = fmaf(z2, poly, 0.4f);
    poly = fmaf(z2, poly, 0.66666666666666667f);
    poly = fmaf(z2, poly, 2.0f);
    return fma((double)e, 0.69314718055994531, (double)(z * poly));
}

// ---------------------------------------------------------------------------
// Sharp read noise (a > A_RECUR_MAX): the window holds a handful of terms; each
// log-summand relative to the one at k0 is formed directly,
//   lw_k = -a((k-c)^2 - (k0-c)^2) + (k - k0) log mu - sum_{j in (k0, k]} log j,
// and both sums are max-free (every lw_k <= ~0 near the mode).
// ---------------------------------------------------------------------------
__device__ inline double lgamma_diff(int k, int k0) {   // lgamma(k+1) - lgamma(k0+1)
    double s = 0.0;
    if (k > k0) for (int j = k0 + 1; j <= k; ++j) s += log((double)j);
    else for (int j = k + 1; j <= k0; ++j) s -= log((double)j);
    return s;
}

__device__ __noinline__ double delta_ell_sharp(float d, float lmu, float lx, Window win, PixConst pc) {
    int k0 = (int)rintf(fmaxf(pc.c, 0.0f));
    k0 = k0 < win.lo ? win.lo : (k0 > win.hi ? win.hi : k0);
    const double a = 0.5 * (double)pc.a2, c = pc.c, lmd = (double)lmu;
    double s0 = 0.0, s1 = 0.0;
    for (int k = win.lo; k <= win.hi; ++k) {
        const double lw = -a * ((k - c) * (k - c) - (k0 - c) * (k0 - c)) + (k - k0) * lmd - lgamma_diff(k, k0);
        s0 += exp_wide(lw);
        s1 += exp_wide(lw + (k - k0) * (double)lx);
    }
    return -(double)d + (double)k0 * (double)lx + log_ratio(s1, s0);
}

// ---------------------------------------------------------------------------
// Local series of one pixel's log-likelihood (used by the block-series scan).
// With v = y/mu, ell(mu + y) - ell(mu) = -y + log E_mu[(1 + v)^phi], the
// expectation under the photon-count posterior at mu.  As a function of mu the
// pixel factor sum_k exp(-a(k - c)^2) mu^k / k! is exp(-a c^2) times the image
// of exp(z), z = mu exp(2ac), under the multiplier sequence exp(-a k^2)
// (Laguerre); by the Polya-Schur theorem it has only real negative zeros, so
//   log E[(1 + v)^phi] = sum_i log(1 + beta_i v),   0 < beta_i < 1,
// and its Taylor coefficients h_j = (-1)^(j+1) sum_i beta_i^j / j give, after
// order J, a remainder of at most  s2 |v|^(J+1) / ((J + 1)(1 - |v|))  with
// s2 = sum_i beta_i^2 = E[phi] - Var[phi] = -2 h_2.
//
// series_at() evaluates h_1..h_4 at mu exactly (up to rounding) from the same
// phi window as delta_ell: Horner's rule from the window top on the degree-4
// polynomial S(v) = sum_k (W_k / W_lo)(1 + v)^(k - lo), then the power-series
// logarithm of S(v)/S(0) plus lo log(1 + v).  Returned, in y-units:
//   ell(mu + y) - ell(mu) = b1 y + b2 y^2 + b3 y^3 + b4 y^4,
//   b1 = h1/mu - 1, bj = hj/mu^j,
// and the radius R = u mu, the largest |y| whose bound stays below
// SERIES_TAU / 2 (u <= 1/2, so mu + y > 0 inside it).  R = 0 (always
// evaluate directly) for sharp read noise, an unusable window or mu <= 0.
// ---------------------------------------------------------------------------
constexpr float SERIES_TAU = 3e-9f;

struct Series { float4 b; float R; };

// Series of the pixel at mean mu from the window polynomial
// A(v) = sum_{k > lo} (W_k / W_lo)(1 + v)^(k - lo) (coefficients A0..A4).
__device__ inline Series series_finish(double A0, double A1, double A2, double A3, double A4, int lo, float mu) {
    Series out;
    const double iS = 1.0 / (1.0 + A0);
    const double s1 = A1 * iS, s2 = A2 * iS, s3 = A3 * iS, s4 = A4 * iS;
    // log(1 + s1 v + s2 v^2 + ...): h_j = s_j - (1/j) sum_{i<j} i h_i s_{j-i}
    const double h1 = s1;
    const double h2 = s2 - 0.5 * h1 * s1;
    const double h3 = s3 - (h1 * s2 + 2.0 * h2 * s1) * (1.0 / 3.0);
    const double h4 = s4 - 0.25 * (h1 * s3 + 2.0 * h2 * s2 + 3.0 * h3 * s1);
    const double L = (double)lo;                     // + lo log(1 + v)
    const double g1 = h1 + L, g2 = h2 - 0.5 * L, g3 = h3 + L * (1.0 / 3.0), g4 = h4 - 0.25 * L;
    const double im = 1.0 / (double)mu, im2 = im * im;
    out.b = make_float4((float)(g1 * im - 1.0), (float)(g2 * im2), (float)(g3 * im2 * im), (float)(g4 * im2 * im2));
    // radius: u0 = (tau/2 * 5 / s2)^(1/5) solves s2 u^5 / 5 = tau/2; the factor
    // (1 - u0)^(1/5) makes room for the 1/(1 - u) of the bound
    const float s2v = fmaxf((float)(-2.0 * g2), 1e-30f);
    float u = __builtin_amdgcn_exp2f(0.2f * __builtin_amdgcn_logf(2.5f * SERIES_TAU * __builtin_amdgcn_rcpf(s2v)));
    u = fminf(u, 0.5f);
    u *= __builtin_amdgcn_exp2f(0.2f * __builtin_amdgcn_logf(1.0f - u));
    out.R = u * mu;
    return out;
}

// ---------------------------------------------------------------------------
// EMCCD pixel: photoelectrons phi ~ Poisson(mu), the multiplication register's
// output x ~ Gamma(phi, 1) (photon units) for phi >= 1 and x = 0 for phi = 0,
// reading w = o + G x with read noise on the zero-photon reading.  With
// c = (w - o)/G and A = Normal(w; o, sigma^2),
//   L(mu) = e^-mu [ A + [c > 0] (e^-c / G) sqrt(mu / c) I_1(2 sqrt(mu c)) ]
// (the photoelectron sum in closed form).  Per-pixel record (c, -1, log A,
// -c - log G): the -1 in place of 2a marks the model; -c - log G is -inf for
// c <= 0, where no photoelectron can have been amplified.
// ---------------------------------------------------------------------------
// log I_1(z), z > 0, in double: the power series
//   I_1(z) = sum_k (z/2)^(2k+1) / (k! (k+1)!)
// for z < 24 (summed until a term falls below 1e-17 of the sum), and for
// z >= 24 the asymptotic expansion (Abramowitz & Stegun 9.7.1, order 1)
//   I_1(z) = e^z / sqrt(2 pi z) sum_k a_k,  a_0 = 1,
//   a_k = -a_(k-1) (4 - (2k - 1)^2) / (8 k z),
// whose terms fall over the first 2z of them, truncated below 1e-17.  Both
// run four terms per step with the step's reciprocals formed off the chain of
// products (hardware reciprocal and one Newton step, full double accuracy),
// so the chain is multiplies and adds only; the tolerance is checked once per
// step (the extra terms of the last step only add more of the exact sum).
__device__ inline double rcp_nr(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return r * fma(-x, r, 2.0);
}

__device__ inline double log_i1(double z) {
    if (z < 24.0) {
        const double h = 0.5 * z, h2 = h * h;
        double t = h, s = h;
#pragma unroll 1
        for (int k = 0; k < 200; k += 4) {
            double q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = h2 * rcp_nr((double)(k + u + 1) * (double)(k + u + 2));
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                t *= q[u];
                s += t;
            }
            if (t < 1e-17 * s) break;
        }
        return log(s);
    }
    const double iz8 = 0.125 / z;
    double a = 1.0, s = 1.0;
#pragma unroll 1
    for (int k = 1; k < 48; k += 4) {
        double q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double m = (double)(2 * (k + u) - 1);
            q[u] = (m * m - 4.0) * iz8 * rcp_nr((double)(k + u));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a *= q[u];
            s += a;
        }
        if (fabs(a) < 1e-17 * s) break;
    }
    return z - 0.5 * log(6.283185307179586 * z) + log(s);
}

// log(e^a + e^b) for finite a, b that may be -inf.
__device__ inline double lse2(double a, double b) {
    const double m = fmax(a, b);
    return m + log1p(exp(-fabs(a - b)));
}

// log L(mu) + mu of an EMCCD pixel from its record fields: log A and
// lB = -c - log G, mu > 0.
__device__ inline double emccd_lse(double mu, double c, double lA, double lB) {
    if (!(c > 0.0)) return lA;
    return lse2(lA, lB + 0.5 * log(mu / c) + log_i1(2.0 * sqrt(mu * c)));
}

// ell(mu + d) - ell(mu) of an EMCCD pixel (NaN when mu + d <= 0).
__device__ inline double delta_ell_emccd(float mu, float d, const PixConst& pc) {
    const double m0 = (double)mu, m1 = (double)mu + (double)d;
    if (!(m1 > 0.0) || !(m0 > 0.0)) return __builtin_nan("");
    if (d == 0.0f) return 0.0;
    if (!(pc.c > 0.0f)) return -(double)d;
    return (emccd_lse(m1, pc.c, pc.L0, pc.iB) - emccd_lse(m0, pc.c, pc.L0, pc.iB)) - (double)d;
}

// ---------------------------------------------------------------------------
// Likelihood change of one footprint pixel:
//   ell(mu + d) - ell(mu) = -d + log( sum_k W_k x^k / sum_k W_k ),  x = 1 + d/mu,
// i.e. the log of the mean of x^phi under the photon-count posterior at mu.
// Both sums run over one window by Horner's rule from the top (normalised at
// the window's lower end, so x^k -> x^(k - lo)), in double precision:
//   acc0 <- r_k (1 + acc0),  acc1 <- x r_k (1 + acc1),  r_k = G_k / (k + 1),
//   G_k = mu exp(-a(2k + 1 - 2c)),  G_{k-1} = G_k exp(2a).
// For a <= A_RECUR_MAX the window's summands span far less than the double
// range (TAIL_T nats deep plus a bracket of a few photons), so the
// normalisation at lo cannot overflow.  Returns NaN when mu + d <= 0 or on
// overflow (the caller then rejects).  inv_tab[k] = 1/k for k < INV_TABLE.
// ---------------------------------------------------------------------------
// With ANCHOR, the same window also yields the local series at mu + d (the
// tilted weights W_k x^k are the posterior weights there), for the caller to
// install if the move is accepted; next->R = 0 where no series is formed.
// TABLE: 1/(k+1) from inv_tab (staged in LDS by the caller), else computed
// (recip4), which keeps memory latency out of the recurrence when no table
// fits in LDS.
template <bool ANCHOR, bool TABLE = true>
__device__ inline double delta_ell_t(float mu, float d, const PixConst& pc, const double* inv_tab, int& nterms,
                                     Series* next) {
    if (ANCHOR) {
        next->R = 0.0f;
        next->b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    const float mu1 = mu + d;
    if (!(mu1 > 0.0f) || !(mu > 0.0f)) return __builtin_nan("");
    if (d == 0.0f) return 0.0;
    const float t = d * fast_rcp(mu);             // relative change
    const float lx = log1p_k(t);                  // log x
    const float lmu = fast_ln(mu);
    const Window win = phi_window(lmu + fminf(lx, 0.0f), lmu + fmaxf(lx, 0.0f), pc);
    if (!win.ok) return __builtin_nan("");
    nterms += win.hi - win.lo + 1;                // the window's terms (work measure)
    if (pc.a2 > 2.0f * A_RECUR_MAX) return delta_ell_sharp(d, lmu, lx, win, pc);
    // The recurrence runs in steps of four terms: the window is widened to a
    // multiple of four (downwards while that stays >= 0, else upwards).  Extra
    // summands only add more of the exact sum.
    int lo = win.lo, hi = win.hi;
    const int n4 = (hi - lo + 3) & ~3;
    lo = hi - n4;
    if (lo < 0) { hi -= lo; lo = 0; }
    const double x = 1.0 + (double)t;
    const double qi = exp_small(pc.a2);           // exp(2a), the ratio of successive G
    const int k_top = hi - 1;
    // |exponent| <= 2 A_RECUR_MAX (2^20 + 1): within exp_wide_b's range
    double G = (double)mu * exp_wide_b(-(double)pc.a2 * ((double)k_top + 0.5 - (double)pc.c));
    double acc0 = 0.0, acc1 = 0.0;
    double A0 = 0.0, A1 = 0.0, A2 = 0.0, A3 = 0.0, A4 = 0.0;   // series polynomial at mu + d
    if (!TABLE || hi < INV_TABLE) {
        const double* iv = inv_tab + hi;          // iv[-i] = 1 / (hi - i)
#pragma unroll 1
        for (int i = 0; i < n4; i += 4) {
            double cv[4];
            if (TABLE) {
#pragma unroll
                for (int u = 0; u < 4; ++u) cv[u] = iv[-(i + u)];
            } else {
                recip4(hi - i, cv);                   // hi - i - 3 >= lo + 1 >= 1
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double r = G * cv[u];
                G *= qi;
                acc0 = fma(r, acc0, r);
                const double rx = r * x;
                acc1 = fma(rx, acc1, rx);
                if (ANCHOR) {
                    const double T0 = A0 + 1.0;
                    A4 = rx * (A4 + A3);
                    A3 = rx * (A3 + A2);
                    A2 = rx * (A2 + A1);
                    A1 = rx * (A1 + T0);
                    A0 = rx * T0;
                }
            }
        }
    } else {
#pragma unroll 1
        for (int k = k_top; k >= lo; --k) {
            const double r = G / (double)(k + 1);
            G *= qi;
            acc0 = fma(r, acc0, r);
            const double rx = r * x;
            acc1 = fma(rx, acc1, rx);
            if (ANCHOR) {
                const double T0 = A0 + 1.0;
                A4 = rx * (A4 + A3);
                A3 = rx * (A3 + A2);
                A2 = rx * (A2 + A1);
                A1 = rx * (A1 + T0);
                A0 = rx * T0;
            }
        }
    }
    if (ANCHOR) *next = series_finish(A0, A1, A2, A3, A4, lo, mu + d);
    // log((1 + acc1)/(1 + acc0)): the sums are normalised at the window's low
    // end and may exceed the FP32 range, so the ratio stays in double.
    return fma((double)lo, (double)lx, log_ratio(1.0 + acc1, 1.0 + acc0) - (double)d);
}

__device__ inline double delta_ell(float mu, float d, const PixConst& pc, const double* inv_tab, int& nterms) {
    return delta_ell_t<false>(mu, d, pc, inv_tab, nterms, nullptr);
}

// The same without a reciprocal table.
__device__ inline double delta_ell_notab(float mu, float d, const PixConst& pc, int& nterms) {
    return delta_ell_t<false, false>(mu, d, pc, nullptr, nterms, nullptr);
}

// A direct evaluation whose series at mu + d is formed only once the move is
// accepted.  delta_ell_keep returns what delta_ell_t<false, false> returns and
// keeps what the window's recurrence needs beyond (mu, d); series_kept(k, mu,
// d) then recomputes x = 1 + d / mu and exp(2a) by the same operations, runs
// the same terms (the products of the ANCHOR pass, in its order, so the series
// is bit-identical to that pass's) and returns the series at mu + d, with
// R = 0 where the evaluation forms none (no move, a rejected window, sharp read
// noise).  A rejected move, about half of them, skips the series' work: the
// polynomial recurrence is two thirds of each term's operations.  The kept
// state is five registers, as many as the series it replaces.
struct DirectKeep {
    double G;    // G at the window top
    int hi, n4;  // window [hi - n4, hi), widened to a multiple of four terms; n4 < 0: no series
    float a2;    // 2a of the pixel
};

__device__ inline double delta_ell_keep(float mu, float d, const PixConst& pc, int& nterms, DirectKeep& k) {
    k.n4 = -1;
    const float mu1 = mu + d;
    if (!(mu1 > 0.0f) || !(mu > 0.0f)) return __builtin_nan("");
    if (d == 0.0f) return 0.0;
    const float t = d * fast_rcp(mu);
    const float lx = log1p_k(t);
    const float lmu = fast_ln(mu);
    const Window win = phi_window(lmu + fminf(lx, 0.0f), lmu + fmaxf(lx, 0.0f), pc);
    if (!win.ok) return __builtin_nan("");
    nterms += win.hi - win.lo + 1;
    if (pc.a2 > 2.0f * A_RECUR_MAX) return delta_ell_sharp(d, lmu, lx, win, pc);
    int lo = win.lo, hi = win.hi;
    const int n4 = (hi - lo + 3) & ~3;
    lo = hi - n4;
    if (lo < 0) { hi -= lo; lo = 0; }
    const double x = 1.0 + (double)t;
    const double qi = exp_small(pc.a2);
    double G = (double)mu * exp_wide_b(-(double)pc.a2 * ((double)(hi - 1) + 0.5 - (double)pc.c));
    k.G = G;
    k.hi = hi;
    k.n4 = n4;
    k.a2 = pc.a2;
    // Four Horner steps acc <- (G_u / n_u)(1 + acc) at a time (n_u = hi - i - u,
    // G_u = G qi^u) over their common denominator N = n0 n1 n2 n3:
    //   acc <- G3 [n2 n1 n0 + G2 (n1 n0 + G1 (n0 + G0 (1 + acc)))] / N,
    // one reciprocal per four terms and no per-term one (every quantity is
    // positive, so nothing cancels).  The terms are those of delta_ell_t's
    // recurrence; series_kept forms the per-term reciprocals its series needs.
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 1
    for (int i = 0; i < n4; i += 4) {
        const double n0 = (double)(hi - i), n1 = n0 - 1.0, n2 = n0 - 2.0, n3 = n0 - 3.0;   // n3 >= lo + 1 >= 1
        const double p10 = n1 * n0, p210 = n2 * p10, N = n3 * p210;
        double iN = __builtin_amdgcn_rcp(N);
        iN = fma(iN, fma(-N, iN, 1.0), iN);
        const double g0 = G, g1 = g0 * qi, g2 = g1 * qi, g3 = g2 * qi;
        G = g3 * qi;
        double t = fma(g0, acc0, g0) + n0;
        t = fma(g1, t, p10);
        t = fma(g2, t, p210);
        acc0 = (g3 * t) * iN;
        const double x0 = g0 * x, x1 = g1 * x, x2 = g2 * x, x3 = g3 * x;
        t = fma(x0, acc1, x0) + n0;
        t = fma(x1, t, p10);
        t = fma(x2, t, p210);
        acc1 = (x3 * t) * iN;
    }
    return fma((double)lo, (double)lx, log_ratio(1.0 + acc1, 1.0 + acc0) - (double)d);
}

__device__ inline Series series_kept(const DirectKeep& k, float mu, float d) {
    Series out;
    out.R = 0.0f;
    out.b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (k.n4 < 0) return out;
    const float t = d * fast_rcp(mu);
    const double x = 1.0 + (double)t;
    const double qi = exp_small(k.a2);
    double G = k.G;
    double A0 = 0.0, A1 = 0.0, A2 = 0.0, A3 = 0.0, A4 = 0.0;
#pragma unroll 1
    for (int i = 0; i < k.n4; i += 4) {
        double cv[4];
        recip4(k.hi - i, cv);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double r = G * cv[u];
            G *= qi;
            const double rx = r * x;
            const double T0 = A0 + 1.0;
            A4 = rx * (A4 + A3);
            A3 = rx * (A3 + A2);
            A2 = rx * (A2 + A1);
            A1 = rx * (A1 + T0);
            A0 = rx * T0;
        }
    }
    return series_finish(A0, A1, A2, A3, A4, k.hi - k.n4, mu + d);
}

// Likelihood change of one footprint pixel for the camera the kernel was
// instantiated for (EM: EMCCD reading, one closed-form term; else sCMOS).
template <bool EM>
__device__ inline double delta_pix(float mu, float d, const PixConst& pc, const double* inv_tab, int& nterms) {
    if constexpr (EM) {
        ++nterms;
        return delta_ell_emccd(mu, d, pc);
    } else {
        return delta_ell(mu, d, pc, inv_tab, nterms);
    }
}

__device__ inline Series series_at(float mu, const PixConst& pc, int& nterms) {
    Series out;
    out.b = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    out.R = 0.0f;
    if (!(mu > 0.0f) || pc.a2 > 2.0f * A_RECUR_MAX || pc.a2 < 0.0f) return out;   // < 0: EMCCD pixel
    const float lmu = fast_ln(mu);
    const Window win = phi_window(lmu, lmu, pc);
    if (!win.ok) return out;
    nterms += win.hi - win.lo + 1;
    // the window widened to a multiple of four terms, as in delta_ell_t
    int lo = win.lo, hi = win.hi;
    const int n4 = (hi - lo + 3) & ~3;
    lo = hi - n4;
    if (lo < 0) { hi -= lo; lo = 0; }
    const double qi = exp_small(pc.a2);
    const int k_top = hi - 1;
    double G = (double)mu * exp_wide_b(-(double)pc.a2 * ((double)k_top + 0.5 - (double)pc.c));
    // A(v) <- r_k (1 + v)(1 + A(v)), coefficients of v^0..v^4, descending so
    // that each update reads the previous step's lower coefficient
    double A0 = 0.0, A1 = 0.0, A2 = 0.0, A3 = 0.0, A4 = 0.0;
#pragma unroll 1
    for (int i = 0; i < n4; i += 4) {
        double cv[4];
        recip4(hi - i, cv);                           // 1/(k+1) for k = k_top - i - u
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double r = G * cv[u];
            G *= qi;
            const double T0 = A0 + 1.0;
            A4 = r * (A4 + A3);
            A3 = r * (A3 + A2);
            A2 = r * (A2 + A1);
            A1 = r * (A1 + T0);
            A0 = r * T0;
        }
    }
    return series_finish(A0, A1, A2, A3, A4, lo, mu);
}

// Change of the series between displacements y0 = D and y1 = D + d from the
// anchor, as d times the divided difference of the polynomial (Horner on both
// points at once), so it stays proportional to d without cancellation.
__device__ inline float series_delta(float4 b, float D, float d) {
    const float y1 = D + d;
    float q = b.w;
    float p = fmaf(b.w, D, b.z);
    q = fmaf(q, y1, p);
    p = fmaf(p, D, b.y);
    q = fmaf(q, y1, p);
    p = fmaf(p, D, b.x);
    q = fmaf(q, y1, p);
    return d * q;
}

}  // namespace bdc
