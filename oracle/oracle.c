/*
 * oracle.c -- FP64 CPU oracle for the Bayesian-deconvolution posterior sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg load it.  It shares no source with the GPU library: its Philox
 * generator, its likelihood, its convolution and its schedules are written
 * here, separately, from the paper and the published definitions.
 *
 * What it computes (paper, Methods):
 *   - expected image    mu_n = sum_m P[n-m] rho_m              (Eqs. 1-2,
 *     object lattice = pixel lattice, zero outside the frame), or, with k x k
 *     object cells per pixel, the PSF-blurred object on the object lattice
 *     summed over each pixel's cells (orc_forward_sub)
 *   - EMCCD reading     Poisson photoelectrons, Gamma(phi, 1) multiplication,
 *     read noise on the zero-photon reading (Discussion; orc_loglik_emccd)
 *   - pixel likelihood  L_n(mu) = sum_{phi>=0} Normal(w_n; G_n phi + o_n, s_n^2)
 *                                       * Poisson(phi; mu)      (Eqs. 3-6)
 *   - posterior         prod_n L_n(mu_n(rho)) * p(rho)          (Eq. 9) with
 *     a separable prior (flat on (0, inf) or Gamma(a, b)) or the Dirichlet-OTF
 *     prior of Eqs. 7-8 read per chunk: one Dirichlet on the normalised
 *     spectrum modulus of each B x B block of the block-phase scan (see
 *     orc_chunk_logprior)
 *   - sampler           Metropolis-within-Gibbs over a systematic scan of
 *     colour groups (pixels of one group have disjoint PSF footprints, the
 *     locality argument of "Parallelization Technique"), log-normal random
 *     walk proposals, accept iff log u < Delta.
 *
 * Everything is double precision.  The phi-sum is truncated to a window that
 * provably holds all but exp(-72) of the mass (see loglik_pixel), which the
 * tests cross-check against a 50-digit full sum.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), implemented from that paper's
 * description; counter = (pixel, sweep, chain, stream), key = (seed_lo,
 * seed_hi).  Streams: 0 proposal normal, 1 accept uniform, 2 initial state,
 * 3 block-proposal normals, 4 block accept uniform.
 *
 * Block independence move (the learned proposal of the GPU library): a
 * Metropolis-Hastings step on a 16 x 16 block of object pixels with an
 * independent log-normal proposal per pixel; see orc_block_pass.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t a_hi = (uint32_t)(pa >> 32), a_lo = (uint32_t)pa;
        uint32_t b_hi = (uint32_t)(pb >> 32), b_lo = (uint32_t)pb;
        uint32_t y0 = b_hi ^ x1 ^ k0;
        uint32_t y1 = b_lo;
        uint32_t y2 = a_hi ^ x3 ^ k1;
        uint32_t y3 = a_lo;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;   /* Weyl sequence key schedule */
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Vector form for the tests: n counters given as 4 words each. */
void orc_philox_many(const uint32_t* ctrs, int64_t n, uint32_t key0, uint32_t key1, uint32_t* out)
{
    uint32_t key[2] = {key0, key1};
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * i, key, out + 4 * i);
}

/* Open-interval uniform from the top 23 bits of a word: ((x >> 9) + 1/2) * 2^-23. */
static double u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

static void draw(uint64_t seed, uint32_t m, uint32_t t, uint32_t chain, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {m, t, chain, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Box-Muller normal from words 0 and 1 of one Philox block. */
double orc_normal(uint64_t seed, uint32_t m, uint32_t t, uint32_t chain, uint32_t stream)
{
    uint32_t r[4];
    draw(seed, m, t, chain, stream, r);
    double u1 = u01(r[0]), u2 = u01(r[1]);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

double orc_uniform(uint64_t seed, uint32_t m, uint32_t t, uint32_t chain, uint32_t stream)
{
    uint32_t r[4];
    draw(seed, m, t, chain, stream, r);
    return u01(r[0]);
}

/* ------------------------------------------------------------------------ */
/* Likelihood of one pixel (Eqs. 3-6)                                        */
/* ------------------------------------------------------------------------ */

/* lgamma(k + 1) for small integers, filled once (before any parallel region). */
#define LGAMMA_TABLE 65536
static double g_lgamma1[LGAMMA_TABLE];
static int g_lgamma_ready = 0;

void orc_prepare(void)
{
    if (g_lgamma_ready) return;
    for (int k = 0; k < LGAMMA_TABLE; ++k) {
        int sg;
        g_lgamma1[k] = lgamma_r((double)k + 1.0, &sg);
    }
    g_lgamma_ready = 1;
}

static double lfact(long k)
{
    if (k < LGAMMA_TABLE) return g_lgamma1[k];
    int sg;
    return lgamma_r((double)k + 1.0, &sg);
}

/*
 * log L_n(mu) = log sum_phi Normal(w; G phi + o, sig^2) Poisson(phi; mu).
 *
 * With c = (w - o)/G and a = G^2/(2 sig^2) the log of a summand is
 *   tau(phi) = -a (phi - c)^2 - lgamma(phi + 1) + phi log mu - mu - log(sqrt(2 pi) sig).
 * tau is concave in phi.  tau' >= 0 for phi <= min(c, mu - 1) and tau' <= 0
 * for phi >= max(c, mu) (digamma(x+1) lies between log(x+1/2) and log(x+1)),
 * so the mode lies in [min(c, mu-1), max(c, mu)], and tau'' <= -2a, so a
 * summand at distance d beyond that bracket is below the largest one by at
 * least exp(-a d^2).  With D = 12 sig/G + 12, a D^2 >= 72: the window
 * [min(c, mu-1) - D, max(c, mu) + D] keeps all but ~e^-72 of the sum.
 * Combined by a max-shifted log-sum-exp.  mu = 0 leaves the phi = 0 term only.
 */
double orc_loglik_pixel(double w, double G, double o, double sig, double mu)
{
    const double c = (w - o) / G;
    const double a = G * G / (2.0 * sig * sig);
    const double lnorm = -0.5 * log(2.0 * M_PI * sig * sig);
    if (!(mu > 0.0)) return lnorm - a * c * c;
    const double D = 12.0 * sig / G + 12.0;
    double lo_d = fmin(c, mu - 1.0) - D;
    double hi_d = fmax(c, mu) + D;
    long lo = lo_d > 0.0 ? (long)floor(lo_d) : 0;
    long hi = (long)ceil(hi_d);
    if (hi < lo) hi = lo;
    const double lmu = log(mu);
    double stackbuf[512];
    double* tau = (hi - lo + 1 <= 512) ? stackbuf : (double*)malloc((size_t)(hi - lo + 1) * sizeof(double));
    double mx = -INFINITY;
    for (long k = lo; k <= hi; ++k) {
        double d = (double)k - c;
        double tk = -a * d * d - lfact(k) + (double)k * lmu;
        tau[k - lo] = tk;
        if (tk > mx) mx = tk;
    }
    double s = 0.0;
    for (long k = lo; k <= hi; ++k) s += exp(tau[k - lo] - mx);
    if (tau != stackbuf) free(tau);
    return lnorm - mu + mx + log(s);
}

/*
 * EMCCD pixel (Discussion: the electron-multiplication stage as an additional
 * intermediate random variable).  Photoelectrons phi ~ Poisson(mu); the
 * multiplication register turns phi >= 1 of them into x ~ Gamma(phi, 1) in
 * photon units (the high-gain limit of the cascade, mean phi) and leaves
 * x = 0 for phi = 0; the reading is w = o + G x, with the Gaussian read noise
 * sig carrying the zero-photon reading (w ~ Normal(o, sig^2) for phi = 0),
 * beside which it is negligible once the register has amplified a photon.
 * With c = (w - o)/G:
 *   L(mu) = e^-mu Normal(w; o, sig^2)
 *         + [c > 0] sum_{phi >= 1} Poisson(phi; mu) Gamma(c; phi, 1) / G.
 * The log-summand of phi >= 1,
 *   t(phi) = phi log(mu c) - lgamma(phi + 1) - lgamma(phi) - mu - c - log c - log G,
 * is concave in phi; successive summands have the ratio mu c / (phi (phi + 1)),
 * so the largest lies within one of m = sqrt(mu c), and over the half-width
 * D = 16 sqrt(m + 1) + 16 on either side of m the summands fall by
 * sum 2 log(phi / m) > 72 nats (at every m; e.g. about 210 at m = 100 and 220
 * at m = 1): the window [m - D, m + D] keeps all but ~e^-72 of the sum, which
 * the tests check against the closed form of the sum (a modified Bessel
 * function).  Combined by a max-shifted log-sum-exp with the phi = 0 term.
 */
double orc_loglik_emccd(double w, double G, double o, double sig, double mu)
{
    const double c = (w - o) / G;
    const double t0 = -0.5 * log(2.0 * M_PI * sig * sig) - (w - o) * (w - o) / (2.0 * sig * sig) - mu;
    if (!(c > 0.0) || !(mu > 0.0)) return t0;
    const double m = sqrt(mu * c);
    const double D = 16.0 * sqrt(m + 1.0) + 16.0;
    long lo = (long)floor(m - D), hi = (long)ceil(m + D);
    if (lo < 1) lo = 1;
    const double lmc = log(mu * c), base = -mu - c - log(c) - log(G);
    double mx = t0;
    for (long k = lo; k <= hi; ++k) {
        const double tk = (double)k * lmc - lfact(k) - lfact(k - 1) + base;
        if (tk > mx) mx = tk;
    }
    double s = exp(t0 - mx);
    for (long k = lo; k <= hi; ++k) s += exp((double)k * lmc - lfact(k) - lfact(k - 1) + base - mx);
    return mx + log(s);
}

void orc_loglik_emccd_many(const double* w, const double* G, const double* o, const double* sig,
                           const double* mu, int64_t n, double* out)
{
    orc_prepare();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_loglik_emccd(w[i], G[i], o[i], sig[i], mu[i]);
}

void orc_loglik_many(const double* w, const double* G, const double* o, const double* sig,
                     const double* mu, int64_t n, double* out)
{
    orc_prepare();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_loglik_pixel(w[i], G[i], o[i], sig[i], mu[i]);
}

/* ------------------------------------------------------------------------ */
/* Forward model (Eqs. 1-2): same-size convolution, zero outside the frame.  */
/* ------------------------------------------------------------------------ */

void orc_forward(const double* rho, int H, int W, const double* psf, int s, double* mu)
{
    const int r = s / 2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int dy = -r; dy <= r; ++dy) {
                int my = y - dy;
                if (my < 0 || my >= H) continue;
                for (int dx = -r; dx <= r; ++dx) {
                    int mx = x - dx;
                    if (mx < 0 || mx >= W) continue;
                    acc += psf[(dy + r) * s + (dx + r)] * rho[(int64_t)my * W + mx];
                }
            }
            mu[(int64_t)y * W + x] = acc;
        }
}

/* Pixel integration over a finer object lattice (Methods, Image Formation
 * Model, Eqs. 1-2, with the object discretised on k x k cells per camera
 * pixel): the blurred irradiance is the convolution of rho with the PSF
 * sampled on the object lattice (zero padding, same size), and pixel (py, px)
 * collects the k x k object cells it covers,
 *   mu[py][px] = sum_{a,b < k} (P (x) rho)[py k + a][px k + b].
 * rho: [k H][k W]; mu: [H][W]. */
void orc_forward_sub(const double* rho, int H, int W, int k, const double* psf, int s, double* mu)
{
    const int Ho = k * H, Wo = k * W;
    double* fine = (double*)malloc((size_t)Ho * Wo * sizeof(double));
    orc_forward(rho, Ho, Wo, psf, s, fine);
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            double acc = 0.0;
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) acc += fine[(int64_t)(py * k + a) * Wo + (px * k + b)];
            mu[(int64_t)py * W + px] = acc;
        }
    free(fine);
}

/* ------------------------------------------------------------------------ */
/* Sampler                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t H, W, s, n_chains;
    int32_t schedule;      /* 1 = pixel-chromatic, 2 = block-phase (four phases),
                              3 = block-phase in nine phases */
    int32_t block;         /* block side B for the block-phase schedules */
    int32_t prior_kind;    /* 0 = flat on (0, inf), 1 = Gamma(shape prior_a, rate prior_b),
                              2 = Dirichlet-OTF prior per block (chunk) of the block-phase scan */
    int32_t burn_in;       /* sweeps with step adaptation; moments afterwards */
    double prior_a, prior_b;
    double log_step0;
    uint64_t seed;
    int32_t camera;        /* 0 = sCMOS (Eqs. 3-6), 1 = EMCCD (orc_loglik_emccd) */
    int32_t sub;           /* object cells per pixel side k (0 or 1: object lattice = pixel
                              lattice); H, W, the frame and the camera maps are the pixel
                              lattice, rho and its moments the (k H) x (k W) object lattice,
                              and the PSF (side s) is sampled on the object lattice */
} orc_config;

typedef struct {
    orc_config cfg;
    double *psf, *w, *G, *o, *sig;      /* normalised PSF, frame and camera maps */
    double *rho, *logstep;              /* [C][k H][k W] (object lattice) */
    double *mu;                         /* [C][H][W] (pixel lattice) */
    double *mean, *m2;                  /* Welford, [C][k H][k W] */
    int64_t n_samples;                  /* post-burn-in sweeps accumulated */
    int64_t t;                          /* next sweep index */
    int64_t *accepts, *proposals;       /* per chain */
    /* schedule: groups of pixels updated together */
    int32_t n_groups;
    int64_t *group_start;               /* n_groups + 1 */
    int32_t *group_pix;                 /* object-cell indices in group order */
    /* Dirichlet-OTF prior (prior_kind 2): concentration alpha of each chunk
     * shape, indexed by (chunk height, chunk width) of the chunk at the frame's
     * bottom / right edge or not: [ey][ex][B*B] */
    double *dir_alpha[2][2];
} orc_ctx;

/* Log-likelihood of frame pixel n at mean mu under the context's camera model. */
static double pix_loglik(const orc_ctx* X, int64_t n, double mu)
{
    return X->cfg.camera == 1 ? orc_loglik_emccd(X->w[n], X->G[n], X->o[n], X->sig[n], mu)
                              : orc_loglik_pixel(X->w[n], X->G[n], X->o[n], X->sig[n], mu);
}

/* Object cells per pixel side, and the sizes of the two lattices. */
static int sub_k(const orc_config* c) { return c->sub > 1 ? c->sub : 1; }
static int64_t n_obj(const orc_config* c) { return (int64_t)sub_k(c) * c->H * sub_k(c) * c->W; }
static int64_t n_pix(const orc_config* c) { return (int64_t)c->H * c->W; }

/* mu of one chain's rho on the pixel lattice. */
static void forward_obs(const orc_ctx* X, const double* rho, double* mu)
{
    if (sub_k(&X->cfg) == 1) orc_forward(rho, X->cfg.H, X->cfg.W, X->psf, X->cfg.s, mu);
    else orc_forward_sub(rho, X->cfg.H, X->cfg.W, sub_k(&X->cfg), X->psf, X->cfg.s, mu);
}

/* ------------------------------------------------------------------------ */
/* Dirichlet-OTF prior (Methods, Prior, Eqs. 7-8), read per chunk             */
/* ------------------------------------------------------------------------ */
/*
 * The prior places a Dirichlet on the normalised modulus of the object's
 * Fourier transform, x_k = |F(rho)_k| / sum_j |F(rho)_j|, with concentration
 * alpha_k = |OTF_k| / sum_j |OTF_j|, OTF = F(PSF) (Eq. 8), the full vectorised
 * spectrum (both k and -k).  Read per chunk: the object is cut into the B x B
 * blocks of the block-phase scan (the paper's padded chunks, Parallelization
 * Technique), the prior is the product of one such Dirichlet per chunk, and
 * the OTF of a chunk is the DFT of the PSF wrapped onto the chunk's grid with
 * its centre at index (0, 0).  alpha_k = 0 (beyond the bandpass) leaves the
 * Dirichlet undefined, so alpha_k <- max(alpha_k, 1e-6 / K), renormalised.
 *
 *   log p(rho_chunk) = lgamma(sum alpha) - sum_k lgamma(alpha_k)
 *                      + sum_k (alpha_k - 1) log x_k.
 */
void orc_dirichlet_alpha(const double* psf, int s, int th, int tw, double* alpha)
{
    const int r = s / 2, K = th * tw;
    double* wr = (double*)calloc((size_t)K, sizeof(double));
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const int y = ((dy % th) + th) % th, x = ((dx % tw) + tw) % tw;
            wr[y * tw + x] += psf[(dy + r) * s + (dx + r)];
        }
    double tot = 0.0;
    for (int ky = 0; ky < th; ++ky)
        for (int kx = 0; kx < tw; ++kx) {
            double re = 0.0, im = 0.0;
            for (int y = 0; y < th; ++y)
                for (int x = 0; x < tw; ++x) {
                    const double a = 2.0 * M_PI * ((double)(ky * y) / th + (double)(kx * x) / tw);
                    re += wr[y * tw + x] * cos(a);
                    im -= wr[y * tw + x] * sin(a);
                }
            alpha[ky * tw + kx] = sqrt(re * re + im * im);
            tot += alpha[ky * tw + kx];
        }
    double tot2 = 0.0;
    for (int k = 0; k < K; ++k) {
        alpha[k] = fmax(alpha[k] / tot, 1e-6 / K);
        tot2 += alpha[k];
    }
    for (int k = 0; k < K; ++k) alpha[k] /= tot2;
    free(wr);
}

/* Modulus of the spectrum of one chunk rho[th][tw] (row stride ld),
 * F_k = sum_m rho_m exp(-2 pi i (ky y / th + kx x / tw)), by the definition;
 * returns sum_k |F_k|. */
static double chunk_modulus(const double* rho, int ld, int th, int tw, double* mod)
{
    double S = 0.0;
    for (int ky = 0; ky < th; ++ky)
        for (int kx = 0; kx < tw; ++kx) {
            double re = 0.0, im = 0.0;
            for (int y = 0; y < th; ++y)
                for (int x = 0; x < tw; ++x) {
                    const double a = 2.0 * M_PI * ((double)((ky * y) % th) / th + (double)((kx * x) % tw) / tw);
                    re += rho[(int64_t)y * ld + x] * cos(a);
                    im -= rho[(int64_t)y * ld + x] * sin(a);
                }
            mod[ky * tw + kx] = sqrt(re * re + im * im);
            S += mod[ky * tw + kx];
        }
    return S;
}

/* log Dirichlet(x; alpha) of one chunk (Eq. 7 at x_k = |F_k| / sum_j |F_j|). */
double orc_chunk_logprior(const double* rho, int ld, int th, int tw, const double* alpha)
{
    const int K = th * tw;
    double* mod = (double*)malloc((size_t)K * sizeof(double));
    const double S = chunk_modulus(rho, ld, th, tw, mod);
    double lp = 0.0, asum = 0.0;
    int sg;
    for (int k = 0; k < K; ++k) {
        asum += alpha[k];
        lp += (alpha[k] - 1.0) * log(mod[k] / S) - lgamma_r(alpha[k], &sg);
    }
    lp += lgamma_r(asum, &sg);
    free(mod);
    return lp;
}

static void chunk_of(const orc_ctx* X, int64_t m, int* y0, int* x0, int* th, int* tw, const double** alpha)
{
    const int B = X->cfg.block, W = X->cfg.W, H = X->cfg.H;
    const int y = (int)(m / W), x = (int)(m % W);
    *y0 = (y / B) * B;
    *x0 = (x / B) * B;
    *th = H - *y0 < B ? H - *y0 : B;
    *tw = W - *x0 < B ? W - *x0 : B;
    *alpha = X->dir_alpha[*th < B][*tw < B];
}

/* Change of the chunk's log prior when pixel m of chain `chain` moves to
 * rho_new: log p(chunk with rho_new) - log p(chunk), the sum over k of
 * (alpha_k - 1)(log x'_k - log x_k); *sabs receives the sum of the absolute
 * values of those terms. */
static double chunk_delta(const orc_ctx* X, int chain, int64_t m, double rho_new, double* sabs)
{
    int y0, x0, th, tw;
    const double* alpha;
    chunk_of(X, m, &y0, &x0, &th, &tw, &alpha);
    const int W = X->cfg.W, K = th * tw;
    const double* rho = X->rho + (int64_t)chain * X->cfg.H * W;
    double* c0 = (double*)malloc((size_t)K * sizeof(double) * 4);
    double *c1 = c0 + K, *m0 = c1 + K, *m1 = m0 + K;
    for (int y = 0; y < th; ++y)
        for (int x = 0; x < tw; ++x) c0[y * tw + x] = c1[y * tw + x] = rho[(int64_t)(y0 + y) * W + (x0 + x)];
    c1[(int)(m / W - y0) * tw + (int)(m % W - x0)] = rho_new;
    const double S0 = chunk_modulus(c0, tw, th, tw, m0);
    const double S1 = chunk_modulus(c1, tw, th, tw, m1);
    double d = 0.0, sa = 0.0;
    for (int k = 0; k < K; ++k) {
        const double term = (alpha[k] - 1.0) * (log(m1[k] / S1) - log(m0[k] / S0));
        d += term;
        sa += fabs(term);
    }
    free(c0);
    if (sabs) *sabs = sa;
    return d;
}

static double log_prior(const orc_config* c, double rho)
{
    if (c->prior_kind == 1) return (c->prior_a - 1.0) * log(rho) - c->prior_b * rho;
    return 0.0;
}

/* Build the scan as a list of pixel groups (all pixels of a group have pairwise
 * disjoint footprints, so their updates commute).
 *
 * Block-phase scans cut the frame into B x B blocks and give block (by, bx) the
 * phase (by mod P, bx mod P), P = 2 (four phases) or 3 (nine); a group is one
 * phase and one position (ly mod s, lx mod s) inside the blocks, phases in
 * order, positions in raster order.  Two pixels of one group either share a
 * block, and then differ by a nonzero multiple of s along some axis, or lie in
 * different blocks of one phase, at least P blocks apart along an axis where
 * the block indices differ, so that their offset along it is at least
 * (P - 1) B + 1 > s - 1 when B >= (s - 1)/(P - 1).  Either way their footprints
 * (side s) are disjoint.  Hence B >= s - 1 for P = 2 and B >= (s - 1)/2 for
 * P = 3. */
static int build_schedule(orc_ctx* X)
{
    const int k = sub_k(&X->cfg);
    const int H = k * X->cfg.H, W = k * X->cfg.W, s = X->cfg.s;
    const int64_t N = (int64_t)H * W;
    /* finer object lattice: object cell (y, x) lies in pixel (y / k, x / k) at
     * phase (y mod k, x mod k); its light reaches the pixels within
     * sp / 2 = floor((s / 2 + k - 1) / k) of its own.  Pixel-chromatic: a group
     * is one cell phase and one pixel position mod sp, so two of its cells lie
     * in pixels at least sp apart along some axis and reach disjoint pixels.
     * Block-phase: the pixel lattice is cut into B x B blocks with the four
     * phases above, and a group is one block phase, one cell phase and one
     * pixel position mod sp inside the blocks (phases, then cell phases, then
     * positions in raster order); two of its cells share a block and lie in
     * pixels a nonzero multiple of sp apart, or lie in same-phase blocks whose
     * pixels are at least B + 1 >= sp apart along some axis. */
    const int sp = 2 * ((s / 2 + k - 1) / k) + 1;
    int ng;
    const int P = X->cfg.schedule == 3 ? 3 : 2;
    if (k > 1) ng = (X->cfg.schedule == 1 ? 1 : 4) * k * k * sp * sp;
    else if (X->cfg.schedule == 1) ng = s * s;
    else ng = P * P * s * s;
    X->n_groups = ng;
    X->group_start = (int64_t*)calloc((size_t)ng + 1, sizeof(int64_t));
    X->group_pix = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    int32_t* gid = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    if (!X->group_start || !X->group_pix || !gid) { free(gid); return ORC_ENOMEM; }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int g;
            if (k > 1 && X->cfg.schedule == 1) {
                g = ((y % k) * k + (x % k)) * sp * sp + ((y / k) % sp) * sp + ((x / k) % sp);
            } else if (k > 1) {
                const int B = X->cfg.block, pyx = y / k, pxx = x / k;
                const int by = pyx / B, bx = pxx / B, ly = pyx - by * B, lx = pxx - bx * B;
                const int bphase = (by % 2) * 2 + (bx % 2), cphase = (y % k) * k + (x % k);
                g = (bphase * k * k + cphase) * sp * sp + (ly % sp) * sp + (lx % sp);
            } else if (X->cfg.schedule == 1) {
                g = (y % s) * s + (x % s);
            } else {
                const int B = X->cfg.block;
                int by = y / B, bx = x / B, ly = y - by * B, lx = x - bx * B;
                int phase = (by % P) * P + (bx % P);
                g = phase * s * s + (ly % s) * s + (lx % s);
            }
            gid[(int64_t)y * W + x] = g;
            X->group_start[g + 1]++;
        }
    for (int g = 0; g < ng; ++g) X->group_start[g + 1] += X->group_start[g];
    int64_t* fill = (int64_t*)malloc((size_t)ng * sizeof(int64_t));
    if (!fill) { free(gid); return ORC_ENOMEM; }
    memcpy(fill, X->group_start, (size_t)ng * sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) X->group_pix[fill[gid[i]]++] = (int32_t)i;  /* ascending */
    free(fill);
    free(gid);
    return ORC_OK;
}

void orc_destroy(orc_ctx* X)
{
    if (!X) return;
    free(X->psf); free(X->w); free(X->G); free(X->o); free(X->sig);
    free(X->rho); free(X->logstep); free(X->mu); free(X->mean); free(X->m2);
    free(X->accepts); free(X->proposals); free(X->group_start); free(X->group_pix);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) free(X->dir_alpha[i][j]);
    free(X);
}

/* Validates, copies the inputs and normalises the PSF.  Camera maps are
 * per-pixel arrays (the caller expands global constants). */
int orc_create(const orc_config* cfg, const double* psf, const double* w, const double* G,
               const double* o, const double* sig, orc_ctx** out)
{
    *out = NULL;
    if (cfg->H < 1 || cfg->W < 1 || cfg->n_chains < 1 || cfg->s < 1 || cfg->s % 2 == 0) return ORC_EINVAL;
    if (cfg->schedule < 1 || cfg->schedule > 3) return ORC_EINVAL;
    if (cfg->sub <= 1 && cfg->schedule == 2 && cfg->block < cfg->s - 1) return ORC_EINVAL;
    if (cfg->schedule == 3 && 2 * cfg->block < cfg->s - 1) return ORC_EINVAL;
    if (cfg->schedule != 1 && cfg->block < 1) return ORC_EINVAL;
    if (cfg->prior_kind < 0 || cfg->prior_kind > 2) return ORC_EINVAL;
    if (cfg->camera != 0 && cfg->camera != 1) return ORC_EINVAL;
    if (cfg->sub < 0 || cfg->sub > 4) return ORC_EINVAL;
    /* a finer object lattice runs the pixel-chromatic scan, or the four-phase
     * block scan with B >= sp - 1 pixels, with a separable prior */
    if (cfg->sub > 1) {
        const int k = cfg->sub, sp = 2 * ((cfg->s / 2 + k - 1) / k) + 1;
        if (cfg->prior_kind == 2 || cfg->schedule == 3) return ORC_EINVAL;
        if (cfg->schedule == 2 && cfg->block < (sp - 1 > 1 ? sp - 1 : 1)) return ORC_EINVAL;
    }
    /* the chunk prior couples the pixels of a block: one pixel per block and group */
    if (cfg->prior_kind == 2 && (cfg->schedule != 2 || cfg->block > cfg->s)) return ORC_EINVAL;
    const int ss = cfg->s * cfg->s;
    double tot = 0.0;
    for (int i = 0; i < ss; ++i) {
        if (!(psf[i] >= 0.0) || !isfinite(psf[i])) return ORC_EINVAL;
        tot += psf[i];
    }
    if (!(tot > 0.0)) return ORC_EINVAL;
    const int64_t N = (int64_t)cfg->H * cfg->W;
    for (int64_t i = 0; i < N; ++i) {
        if (!isfinite(w[i]) || !isfinite(o[i])) return ORC_EINVAL;
        if (!(G[i] > 0.0) || !(sig[i] > 0.0) || !isfinite(G[i]) || !isfinite(sig[i])) return ORC_EINVAL;
    }
    orc_prepare();
    orc_ctx* X = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    if (!X) return ORC_ENOMEM;
    X->cfg = *cfg;
    const int64_t CN = n_obj(cfg) * cfg->n_chains;
    X->psf = (double*)malloc(ss * sizeof(double));
    X->w = (double*)malloc(N * sizeof(double));
    X->G = (double*)malloc(N * sizeof(double));
    X->o = (double*)malloc(N * sizeof(double));
    X->sig = (double*)malloc(N * sizeof(double));
    X->rho = (double*)calloc(CN, sizeof(double));
    X->logstep = (double*)calloc(CN, sizeof(double));
    X->mu = (double*)calloc(N * cfg->n_chains, sizeof(double));
    X->mean = (double*)calloc(CN, sizeof(double));
    X->m2 = (double*)calloc(CN, sizeof(double));
    X->accepts = (int64_t*)calloc(cfg->n_chains, sizeof(int64_t));
    X->proposals = (int64_t*)calloc(cfg->n_chains, sizeof(int64_t));
    if (!X->psf || !X->w || !X->G || !X->o || !X->sig || !X->rho || !X->logstep || !X->mu ||
        !X->mean || !X->m2 || !X->accepts || !X->proposals) { orc_destroy(X); return ORC_ENOMEM; }
    for (int i = 0; i < ss; ++i) X->psf[i] = psf[i] / tot;
    memcpy(X->w, w, N * sizeof(double));
    memcpy(X->G, G, N * sizeof(double));
    memcpy(X->o, o, N * sizeof(double));
    memcpy(X->sig, sig, N * sizeof(double));
    int rc = build_schedule(X);
    if (rc != ORC_OK) { orc_destroy(X); return rc; }
    if (cfg->prior_kind == 2) {
        const int B = cfg->block;
        const int eh = cfg->H % B ? cfg->H % B : B, ew = cfg->W % B ? cfg->W % B : B;
        for (int ey = 0; ey < 2; ++ey)
            for (int ex = 0; ex < 2; ++ex) {
                const int th = ey ? eh : B, tw = ex ? ew : B;
                X->dir_alpha[ey][ex] = (double*)malloc((size_t)th * tw * sizeof(double));
                if (!X->dir_alpha[ey][ex]) { orc_destroy(X); return ORC_ENOMEM; }
                orc_dirichlet_alpha(X->psf, cfg->s, th, tw, X->dir_alpha[ey][ex]);
            }
    }
    *out = X;
    return ORC_OK;
}

/* Initial state: rho0 given ([C][k H][k W], all > 0), or
 * rho_m = max(c_n, 1/2) / k^2 exp(xi_m / 2) for object cell m in pixel n,
 * xi from stream 2 at sweep 0 (one draw per chain and cell). */
int orc_init(orc_ctx* X, const double* rho0)
{
    const int k = sub_k(&X->cfg), Wo = k * X->cfg.W;
    const int64_t N = n_obj(&X->cfg);
    const int C = X->cfg.n_chains;
    for (int ch = 0; ch < C; ++ch)
        for (int64_t m = 0; m < N; ++m) {
            double v;
            if (rho0) {
                v = rho0[ch * N + m];
                if (!(v > 0.0) || !isfinite(v)) return ORC_EINVAL;
            } else {
                const int64_t n = (int64_t)((m / Wo) / k) * X->cfg.W + (m % Wo) / k;
                double c = (X->w[n] - X->o[n]) / X->G[n];
                v = fmax(c, 0.5) / (double)(k * k) *
                    exp(0.5 * orc_normal(X->cfg.seed, (uint32_t)m, 0, (uint32_t)ch, 2));
            }
            X->rho[ch * N + m] = v;
            X->logstep[ch * N + m] = X->cfg.log_step0;
        }
    X->t = 0;
    X->n_samples = 0;
    memset(X->mean, 0, C * N * sizeof(double));
    memset(X->m2, 0, C * N * sizeof(double));
    memset(X->accepts, 0, C * sizeof(int64_t));
    memset(X->proposals, 0, C * sizeof(int64_t));
    return ORC_OK;
}

/* Log-posterior of one chain's state (up to the constant of a flat prior). */
double orc_log_posterior(orc_ctx* X, int chain)
{
    const int H = X->cfg.H, W = X->cfg.W;
    const int64_t N = n_obj(&X->cfg), Np = n_pix(&X->cfg);
    double* mu = (double*)malloc(Np * sizeof(double));
    forward_obs(X, X->rho + chain * N, mu);
    double lp = 0.0;
    for (int64_t n = 0; n < N; ++n) {                 /* N >= Np */
        if (n < Np) lp += pix_loglik(X, n, mu[n]);
        lp += log_prior(&X->cfg, X->rho[chain * N + n]);
    }
    free(mu);
    if (X->cfg.prior_kind == 2) {
        const int B = X->cfg.block;
        for (int y0 = 0; y0 < H; y0 += B)
            for (int x0 = 0; x0 < W; x0 += B) {
                int yy, xx, th, tw;
                const double* alpha;
                chunk_of(X, (int64_t)y0 * W + x0, &yy, &xx, &th, &tw, &alpha);
                lp += orc_chunk_logprior(X->rho + chain * N + (int64_t)y0 * W + x0, W, th, tw, alpha);
            }
    }
    return lp;
}

/* One Metropolis update of object cell m (object lattice k H x k W, k > 1) of
 * one chain at sweep t, with mu current.  The move rho_m -> rho_m + d changes
 * the mean of pixel n by d K_m[n], K_m[n] = sum of the PSF over the offsets
 * from m to the cells of pixel n (Eqs. 1-2 on the finer lattice); Delta sums
 * the likelihood change over those pixels, then the prior and Hastings terms
 * as for a pixel. */
static int update_cell(orc_ctx* X, int chain, int64_t m, int64_t t,
                       double* rec_delta, double* rec_logu, uint8_t* rec_acc, double* rec_sabs)
{
    const int k = sub_k(&X->cfg), H = X->cfg.H, W = X->cfg.W, Ho = k * H, Wo = k * W;
    const int s = X->cfg.s, r = s / 2;
    const int64_t N = n_obj(&X->cfg), Np = n_pix(&X->cfg);
    double* rho = X->rho + chain * N;
    double* mu = X->mu + chain * Np;
    const int y = (int)(m / Wo), x = (int)(m % Wo);
    /* K_m over the pixels that cells within r of m fall in: pixels
     * [(y - r) / k, (y + r) / k] x [(x - r) / k, (x + r) / k], clipped */
    const int py0 = (y - r < 0 ? 0 : y - r) / k, py1 = (y + r >= Ho ? Ho - 1 : y + r) / k;
    const int px0 = (x - r < 0 ? 0 : x - r) / k, px1 = (x + r >= Wo ? Wo - 1 : x + r) / k;
    const int kh = py1 - py0 + 1, kw = px1 - px0 + 1;
    double* K = (double*)calloc((size_t)kh * kw, sizeof(double));
    for (int dy = -r; dy <= r; ++dy) {
        const int cy = y + dy;
        if (cy < 0 || cy >= Ho) continue;
        for (int dx = -r; dx <= r; ++dx) {
            const int cx = x + dx;
            if (cx < 0 || cx >= Wo) continue;
            K[(cy / k - py0) * kw + (cx / k - px0)] += X->psf[(dy + r) * s + (dx + r)];
        }
    }
    const double step = exp(X->logstep[chain * N + m]);
    const double xi = orc_normal(X->cfg.seed, (uint32_t)m, (uint32_t)t, (uint32_t)chain, 0);
    const double rho_old = rho[m];
    const double rho_new = rho_old * exp(step * xi);
    const double delta_rho = rho_new - rho_old;
    double delta = 0.0, sabs = 0.0;
    for (int i = 0; i < kh; ++i)
        for (int j = 0; j < kw; ++j) {
            if (K[i * kw + j] == 0.0) continue;
            const int64_t n = (int64_t)(py0 + i) * W + (px0 + j);
            const double dl = pix_loglik(X, n, mu[n] + delta_rho * K[i * kw + j]) - pix_loglik(X, n, mu[n]);
            delta += dl;
            sabs += fabs(dl);
        }
    delta += log_prior(&X->cfg, rho_new) - log_prior(&X->cfg, rho_old);
    delta += log(rho_new) - log(rho_old);       /* Hastings term of the log-normal walk */
    const double logu = log(orc_uniform(X->cfg.seed, (uint32_t)m, (uint32_t)t, (uint32_t)chain, 1));
    const int acc = isfinite(delta) && (logu < delta);
    if (acc) {
        rho[m] = rho_new;
        for (int i = 0; i < kh; ++i)
            for (int j = 0; j < kw; ++j) mu[(int64_t)(py0 + i) * W + (px0 + j)] += delta_rho * K[i * kw + j];
    }
    free(K);
    if (t < X->cfg.burn_in)
        X->logstep[chain * N + m] += pow((double)t + 1.0, -0.6) * ((double)acc - 0.44);
    if (rec_delta) rec_delta[chain * N + m] = delta;
    if (rec_logu) rec_logu[chain * N + m] = logu;
    if (rec_acc) rec_acc[chain * N + m] = (uint8_t)acc;
    if (rec_sabs) rec_sabs[chain * N + m] = sabs;
    return acc;
}

/* One Metropolis update of pixel m of one chain at sweep t, with mu current.
 * Records Delta, log u and the decision when the pointers are non-null. */
static int update_pixel(orc_ctx* X, int chain, int64_t m, int64_t t,
                        double* rec_delta, double* rec_logu, uint8_t* rec_acc, double* rec_sabs)
{
    if (sub_k(&X->cfg) > 1) return update_cell(X, chain, m, t, rec_delta, rec_logu, rec_acc, rec_sabs);
    const int H = X->cfg.H, W = X->cfg.W, s = X->cfg.s, r = s / 2;
    const int64_t N = (int64_t)H * W;
    double* rho = X->rho + chain * N;
    double* mu = X->mu + chain * N;
    const int y = (int)(m / W), x = (int)(m % W);
    const double step = exp(X->logstep[chain * N + m]);
    const double xi = orc_normal(X->cfg.seed, (uint32_t)m, (uint32_t)t, (uint32_t)chain, 0);
    const double rho_old = rho[m];
    const double rho_new = rho_old * exp(step * xi);
    const double delta_rho = rho_new - rho_old;
    double delta = 0.0, sabs = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
        int ny = y + dy;
        if (ny < 0 || ny >= H) continue;
        for (int dx = -r; dx <= r; ++dx) {
            int nx = x + dx;
            if (nx < 0 || nx >= W) continue;
            int64_t n = (int64_t)ny * W + nx;
            double p = X->psf[(dy + r) * s + (dx + r)];
            double mu_new = mu[n] + delta_rho * p;
            double dl = pix_loglik(X, n, mu_new) - pix_loglik(X, n, mu[n]);
            delta += dl;
            sabs += fabs(dl);
        }
    }
    if (X->cfg.prior_kind == 2) {
        double sp = 0.0;
        delta += chunk_delta(X, chain, m, rho_new, &sp);
        sabs += sp;
    } else {
        delta += log_prior(&X->cfg, rho_new) - log_prior(&X->cfg, rho_old);
    }
    delta += log(rho_new) - log(rho_old);       /* Hastings term of the log-normal walk */
    const double logu = log(orc_uniform(X->cfg.seed, (uint32_t)m, (uint32_t)t, (uint32_t)chain, 1));
    const int acc = isfinite(delta) && (logu < delta);
    if (acc) {
        rho[m] = rho_new;
        for (int dy = -r; dy <= r; ++dy) {
            int ny = y + dy;
            if (ny < 0 || ny >= H) continue;
            for (int dx = -r; dx <= r; ++dx) {
                int nx = x + dx;
                if (nx < 0 || nx >= W) continue;
                mu[(int64_t)ny * W + nx] += delta_rho * X->psf[(dy + r) * s + (dx + r)];
            }
        }
    }
    if (t < X->cfg.burn_in)
        X->logstep[chain * N + m] += pow((double)t + 1.0, -0.6) * ((double)acc - 0.44);
    if (rec_delta) rec_delta[chain * N + m] = delta;
    if (rec_logu) rec_logu[chain * N + m] = logu;
    if (rec_acc) rec_acc[chain * N + m] = (uint8_t)acc;
    if (rec_sabs) rec_sabs[chain * N + m] = sabs;
    return acc;
}

static void run_group(orc_ctx* X, int g, int64_t t, double* rd, double* rl, uint8_t* ra, double* rs)
{
    const int C = X->cfg.n_chains;
    const int64_t b = X->group_start[g], e = X->group_start[g + 1];
    for (int ch = 0; ch < C; ++ch) {
        int64_t acc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : acc)
        for (int64_t i = b; i < e; ++i) acc += update_pixel(X, ch, X->group_pix[i], t, rd, rl, ra, rs);
        X->accepts[ch] += acc;
        X->proposals[ch] += e - b;
    }
}

static void refresh_mu(orc_ctx* X)
{
    const int64_t N = n_obj(&X->cfg), Np = n_pix(&X->cfg);
    for (int ch = 0; ch < X->cfg.n_chains; ++ch) forward_obs(X, X->rho + ch * N, X->mu + ch * Np);
}

static void accumulate_moments(orc_ctx* X)
{
    const int64_t CN = n_obj(&X->cfg) * X->cfg.n_chains;
    X->n_samples += 1;
    const double n = (double)X->n_samples;
    for (int64_t i = 0; i < CN; ++i) {
        double d = X->rho[i] - X->mean[i];
        X->mean[i] += d / n;
        X->m2[i] += d * (X->rho[i] - X->mean[i]);
    }
}

/* n full sweeps.  Each: mu <- P (x) rho from scratch, every group in order,
 * then moments if the sweep index is at or past burn-in.
 * trace_logpost (optional, [n][C]) receives the log-posterior after each sweep. */
int orc_sweeps(orc_ctx* X, int n, double* trace_logpost)
{
    for (int i = 0; i < n; ++i) {
        const int64_t t = X->t;
        refresh_mu(X);
        for (int g = 0; g < X->n_groups; ++g) run_group(X, g, t, NULL, NULL, NULL, NULL);
        if (t >= X->cfg.burn_in) accumulate_moments(X);
        if (trace_logpost)
            for (int ch = 0; ch < X->cfg.n_chains; ++ch)
                trace_logpost[(int64_t)i * X->cfg.n_chains + ch] = orc_log_posterior(X, ch);
        X->t = t + 1;
    }
    return ORC_OK;
}

/* Run groups [g0, g1) of sweep t from the current state (mu is refreshed first
 * when refresh != 0), recording Delta, log u, decisions and sum_n |delta ell_n|
 * ([C][H][W]; untouched pixels keep their previous contents). */
int orc_run_groups(orc_ctx* X, int64_t t, int g0, int g1, int refresh,
                   double* rec_delta, double* rec_logu, uint8_t* rec_acc, double* rec_sabs)
{
    if (g0 < 0 || g1 > X->n_groups || g0 > g1) return ORC_EINVAL;
    if (refresh) refresh_mu(X);
    for (int g = g0; g < g1; ++g) run_group(X, g, t, rec_delta, rec_logu, rec_acc, rec_sabs);
    return ORC_OK;
}

int orc_set_state(orc_ctx* X, const double* rho, const double* logstep, int64_t t)
{
    const int64_t CN = n_obj(&X->cfg) * X->cfg.n_chains;
    for (int64_t i = 0; i < CN; ++i)
        if (!(rho[i] > 0.0) || !isfinite(rho[i])) return ORC_EINVAL;
    memcpy(X->rho, rho, CN * sizeof(double));
    memcpy(X->logstep, logstep, CN * sizeof(double));
    X->t = t;
    return ORC_OK;
}

void orc_get_state(const orc_ctx* X, double* rho, double* logstep, double* mu, int64_t* t)
{
    const int64_t CN = n_obj(&X->cfg) * X->cfg.n_chains;
    if (rho) memcpy(rho, X->rho, CN * sizeof(double));
    if (logstep) memcpy(logstep, X->logstep, CN * sizeof(double));
    if (mu) memcpy(mu, X->mu, n_pix(&X->cfg) * X->cfg.n_chains * sizeof(double));
    if (t) *t = X->t;
}

int32_t orc_n_groups(const orc_ctx* X) { return X->n_groups; }

void orc_group(const orc_ctx* X, int g, int64_t* begin, int64_t* end, const int32_t** pix)
{
    *begin = X->group_start[g];
    *end = X->group_start[g + 1];
    *pix = X->group_pix;
}

void orc_accept_counts(const orc_ctx* X, int64_t* accepts, int64_t* proposals)
{
    for (int ch = 0; ch < X->cfg.n_chains; ++ch) {
        accepts[ch] = X->accepts[ch];
        proposals[ch] = X->proposals[ch];
    }
}

/* Posterior moments.  chain >= 0: that chain's mean and sample variance
 * M2/(n-1).  chain = -1: the pooled sample mean and variance of all C*n draws. */
int orc_moments(const orc_ctx* X, int chain, double* mean, double* var, int64_t* n_out)
{
    const int64_t N = n_obj(&X->cfg);
    const int C = X->cfg.n_chains;
    const int64_t n = X->n_samples;
    *n_out = n;
    if (n < 2) return ORC_EINVAL;
    if (chain >= 0) {
        for (int64_t i = 0; i < N; ++i) {
            mean[i] = X->mean[chain * N + i];
            var[i] = X->m2[chain * N + i] / (double)(n - 1);
        }
        return ORC_OK;
    }
    for (int64_t i = 0; i < N; ++i) {
        double m = 0.0;
        for (int ch = 0; ch < C; ++ch) m += X->mean[ch * N + i];
        m /= C;
        double ss = 0.0;
        for (int ch = 0; ch < C; ++ch) {
            double d = X->mean[ch * N + i] - m;
            ss += X->m2[ch * N + i] + (double)n * d * d;
        }
        mean[i] = m;
        var[i] = ss / (double)(C * n - 1);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Convergence diagnostics (not in the paper)                               */
/* ------------------------------------------------------------------------ */

/* Split-R-hat (Gelman et al., Bayesian Data Analysis 3rd ed., sec. 11.4):
 * each of the C chains (x[c*n + i]) is cut into two halves of length n/2 (the
 * middle draw is dropped when n is odd); with m = 2C sequences of length L,
 * B = L/(m-1) sum_j (mean_j - mean)^2, W = mean_j var_j (unbiased),
 * var+ = (L-1)/L W + B/L, R = sqrt(var+ / W). */
double orc_split_rhat(const double* x, int C, int64_t n)
{
    const int64_t L = n / 2;
    const int m = 2 * C;
    if (L < 2 || m < 2) return NAN;
    double* means = (double*)malloc(m * sizeof(double));
    double* vars = (double*)malloc(m * sizeof(double));
    for (int c = 0; c < C; ++c)
        for (int h = 0; h < 2; ++h) {
            const double* seq = x + (int64_t)c * n + (h == 0 ? 0 : n - L);
            double s = 0.0;
            for (int64_t i = 0; i < L; ++i) s += seq[i];
            double mj = s / L, v = 0.0;
            for (int64_t i = 0; i < L; ++i) v += (seq[i] - mj) * (seq[i] - mj);
            means[2 * c + h] = mj;
            vars[2 * c + h] = v / (L - 1);
        }
    double gm = 0.0, Wv = 0.0;
    for (int j = 0; j < m; ++j) { gm += means[j]; Wv += vars[j]; }
    gm /= m;
    Wv /= m;
    double Bv = 0.0;
    for (int j = 0; j < m; ++j) Bv += (means[j] - gm) * (means[j] - gm);
    Bv *= (double)L / (m - 1);
    free(means);
    free(vars);
    double vplus = (double)(L - 1) / L * Wv + Bv / L;
    return sqrt(vplus / Wv);
}

/* Batch-means Monte Carlo standard error of the mean of x[0..n): n_batches
 * contiguous batches of equal length b = n / n_batches (the tail is dropped);
 * MCSE = sqrt(var(batch means) / n_batches). */
double orc_batch_means_mcse(const double* x, int64_t n, int64_t n_batches)
{
    if (n_batches < 2) return NAN;
    const int64_t b = n / n_batches;
    if (b < 1) return NAN;
    double* bm = (double*)malloc(n_batches * sizeof(double));
    double tot = 0.0;
    for (int64_t k = 0; k < n_batches; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < b; ++i) s += x[k * b + i];
        bm[k] = s / b;
        tot += bm[k];
    }
    const double mean = tot / n_batches;
    double v = 0.0;
    for (int64_t k = 0; k < n_batches; ++k) v += (bm[k] - mean) * (bm[k] - mean);
    v /= (n_batches - 1);
    free(bm);
    return sqrt(v / n_batches);
}


/* ------------------------------------------------------------------------ */
/* Block independence move                                                   */
/* ------------------------------------------------------------------------ */

#define ORC_BS 16

/* Blocks of one colour lie period blocks apart, period = 1 + ceil(2r / 16), so
 * the pixels whose mean a block can change (the block grown by r on each side)
 * never overlap between two blocks of one colour. */
int32_t orc_block_period(int32_t s)
{
    const int r = s / 2;
    return 1 + (2 * r + ORC_BS - 1) / ORC_BS;
}

/* One block.  In u = log rho, with the reference density N(pm_m, ps_m^2) and
 * z = (u - pm_m)/ps_m, every pixel m of the block moves to
 *   z' = sqrt(1 - beta^2) z + beta xi_m,   xi_m ~ N(0, 1) from stream 3 at (m, pass, chain),
 * an AR(1) step that is reversible with respect to the reference (beta = 1:
 * rho' ~ LogNormal(pm, ps^2), independent of rho).  Accept iff
 *   log u < sum_n [ell_n(mu'_n) - ell_n(mu_n)] + sum_m [log p(rho'_m) - log p(rho_m)]
 *           + sum_m [r_m(rho_m) - r_m(rho'_m)],
 * r_m(x) = -log x - (log x - pm_m)^2 / (2 ps_m^2), the reference as a density
 * of rho (Metropolis-Hastings ratio of a reference-reversible proposal),
 * u from stream 4 at (first pixel of the block, pass, chain).  Returns the
 * decision; *delta receives the log acceptance ratio. */
/* With walk > 0 the block instead takes a symmetric random-walk step in
 * u = log rho along the directions the blur removes: every pixel moves by
 * walk * h_m, h = xi - P (x)_B xi, xi_m ~ N(0, 1) from stream 3 at
 * (m, pass, chain) and (P (x)_B xi)_m = sum_{m' in block} P[m - m'] xi_m' the
 * blur of xi restricted to the block's pixels inside the frame.  h is linear
 * in the symmetric xi, so the proposal is symmetric in u and the log
 * acceptance ratio is Delta log pi + sum_m (u'_m - u_m) (the Jacobian of
 * rho = e^u); pm and ps are not used. */
static int block_update(orc_ctx* X, int chain, int by, int bx, int64_t pass, const double* pm, const double* ps,
                        double beta, double walk, double* delta_out, double* sabs_out)
{
    const int H = X->cfg.H, W = X->cfg.W, s = X->cfg.s, r = s / 2;
    const int64_t N = (int64_t)H * W;
    double* rho = X->rho + chain * N;
    double* mu = X->mu + chain * N;
    const int y0 = by * ORC_BS, x0 = bx * ORC_BS;
    const int y1 = y0 + ORC_BS < H ? y0 + ORC_BS : H, x1 = x0 + ORC_BS < W ? x0 + ORC_BS : W;
    const int bh = y1 - y0, bw = x1 - x0;
    double d[ORC_BS * ORC_BS], rp[ORC_BS * ORC_BS], h[ORC_BS * ORC_BS];
    double delta = 0.0, sabs = 0.0;
    if (walk > 0.0) {
        double xi[ORC_BS * ORC_BS];
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x)
                xi[(y - y0) * ORC_BS + (x - x0)] =
                    orc_normal(X->cfg.seed, (uint32_t)((int64_t)y * W + x), (uint32_t)pass, (uint32_t)chain, 3);
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                double b = 0.0;
                for (int yy = y0; yy < y1; ++yy)
                    for (int xx = x0; xx < x1; ++xx) {
                        const int dy = y - yy, dx = x - xx;
                        if (dy < -r || dy > r || dx < -r || dx > r) continue;
                        b += X->psf[(dy + r) * s + (dx + r)] * xi[(yy - y0) * ORC_BS + (xx - x0)];
                    }
                h[(y - y0) * ORC_BS + (x - x0)] = xi[(y - y0) * ORC_BS + (x - x0)] - b;
            }
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) {
                const int64_t m = (int64_t)y * W + x;
                const double lold = log(rho[m]);
                const double lnew = lold + walk * h[(y - y0) * ORC_BS + (x - x0)];
                const double rnew = exp(lnew);
                const double term = log_prior(&X->cfg, rnew) - log_prior(&X->cfg, rho[m]) + (lnew - lold);
                delta += term;
                sabs += fabs(term);
                d[(y - y0) * ORC_BS + (x - x0)] = rnew - rho[m];
                rp[(y - y0) * ORC_BS + (x - x0)] = rnew;
            }
    }
    for (int y = y0; y < y1 && walk <= 0.0; ++y)
        for (int x = x0; x < x1; ++x) {
            const int64_t m = (int64_t)y * W + x;
            const double xi = orc_normal(X->cfg.seed, (uint32_t)m, (uint32_t)pass, (uint32_t)chain, 3);
            const double lold = log(rho[m]);
            const double zo = (lold - pm[m]) / ps[m];
            const double zn = sqrt(1.0 - beta * beta) * zo + beta * xi;
            const double lnew = pm[m] + ps[m] * zn;
            const double rnew = exp(lnew);
            const double lq_old = -lold - 0.5 * zo * zo;
            const double lq_new = -lnew - 0.5 * zn * zn;
            const double term = log_prior(&X->cfg, rnew) - log_prior(&X->cfg, rho[m]) + lq_old - lq_new;
            delta += term;
            sabs += fabs(lq_old) + fabs(lq_new);
            d[(y - y0) * ORC_BS + (x - x0)] = rnew - rho[m];
            rp[(y - y0) * ORC_BS + (x - x0)] = rnew;
        }
    /* region of changed means: the block grown by r, inside the frame */
    const int ry0 = y0 - r > 0 ? y0 - r : 0, ry1 = y1 + r < H ? y1 + r : H;
    const int rx0 = x0 - r > 0 ? x0 - r : 0, rx1 = x1 + r < W ? x1 + r : W;
    const int RH = ry1 - ry0, RWd = rx1 - rx0;
    double* dmu = (double*)malloc(sizeof(double) * (size_t)RH * RWd);
    if (!dmu) return 0;
    for (int ny = ry0; ny < ry1; ++ny)
        for (int nx = rx0; nx < rx1; ++nx) {
            double a = 0.0;
            for (int j = 0; j < bh; ++j)
                for (int i = 0; i < bw; ++i) {
                    const int dy = ny - (y0 + j), dx = nx - (x0 + i);
                    if (dy < -r || dy > r || dx < -r || dx > r) continue;
                    a += d[j * ORC_BS + i] * X->psf[(dy + r) * s + (dx + r)];
                }
            dmu[(ny - ry0) * RWd + (nx - rx0)] = a;
            const int64_t n = (int64_t)ny * W + nx;
            const double dl = pix_loglik(X, n, mu[n] + a) - pix_loglik(X, n, mu[n]);
            delta += dl;
            sabs += fabs(dl);
        }
    const int64_t m0 = (int64_t)y0 * W + x0;
    const double logu = log(orc_uniform(X->cfg.seed, (uint32_t)m0, (uint32_t)pass, (uint32_t)chain, 4));
    const int acc = isfinite(delta) && (logu < delta);
    if (acc) {
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) rho[(int64_t)y * W + x] = rp[(y - y0) * ORC_BS + (x - x0)];
        for (int ny = ry0; ny < ry1; ++ny)
            for (int nx = rx0; nx < rx1; ++nx) mu[(int64_t)ny * W + nx] += dmu[(ny - ry0) * RWd + (nx - rx0)];
    }
    free(dmu);
    if (delta_out) *delta_out = delta;
    if (sabs_out) *sabs_out = sabs;
    return acc;
}

/* One pass of block moves (the reference move, or the walk when walk > 0) at
 * block-pass index `pass`: mu <- P (x) rho, then
 * every block colour (cy, cx) in ascending cy * period + cx (or only colour
 * `colour_only` when >= 0), the blocks of a colour in ascending (by, bx).
 * rec_delta / rec_acc / rec_sabs ([C][blocks of the colour], optional) record
 * the last colour run (rec_sabs: the sum of the absolute values of the terms of
 * Delta, the scale of its rounding).  Returns the number of accepted blocks. */
int64_t orc_block_pass(orc_ctx* X, int64_t pass, int32_t colour_only, const double* pm, const double* ps,
                       double beta, double walk, double* rec_delta, uint8_t* rec_acc, double* rec_sabs,
                       int32_t* n_blocks)
{
    const int H = X->cfg.H, W = X->cfg.W, C = X->cfg.n_chains;
    const int P = orc_block_period(X->cfg.s);
    const int nby = (H + ORC_BS - 1) / ORC_BS, nbx = (W + ORC_BS - 1) / ORC_BS;
    int64_t accepted = 0;
    if (X->cfg.prior_kind == 2) return ORC_EINVAL;      /* 16 x 16 blocks straddle the prior's chunks */
    if (sub_k(&X->cfg) > 1) return ORC_EINVAL;          /* blocks are on the pixel lattice */
    refresh_mu(X);
    for (int k = 0; k < P * P; ++k) {
        if (colour_only >= 0 && k != colour_only) continue;
        const int cy = k / P, cx = k % P;
        int nb = 0;
        for (int by = cy; by < nby; by += P)
            for (int bx = cx; bx < nbx; bx += P) ++nb;
        if (n_blocks) *n_blocks = nb;
        for (int ch = 0; ch < C; ++ch) {
            int64_t acc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : acc)
            for (int b = 0; b < nb; ++b) {
                const int nbx_c = (nbx - cx + P - 1) / P;
                const int by = cy + P * (b / nbx_c), bx = cx + P * (b % nbx_c);
                double dl = 0.0, sa = 0.0;
                const int a = block_update(X, ch, by, bx, pass, pm, ps, beta, walk, &dl, &sa);
                acc += a;
                if (rec_delta) rec_delta[(int64_t)ch * nb + b] = dl;
                if (rec_sabs) rec_sabs[(int64_t)ch * nb + b] = sa;
                if (rec_acc) rec_acc[(int64_t)ch * nb + b] = (uint8_t)a;
            }
            accepted += acc;
        }
    }
    return accepted;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
