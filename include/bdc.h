/*
 * bdc.h -- C ABI of the MI355X (gfx950) posterior sampler for physically
 * motivated Bayesian deconvolution (Hendrix et al., "Re-thinking
 * Richardson-Lucy without Iteration Cutoffs", arXiv:2411.00991).
 *
 * The library samples the posterior over a strictly positive object density
 * rho on the pixel lattice, given one raw sCMOS frame w (ADU), a shift-
 * invariant PSF and per-pixel (or global) camera gain G, offset o and read
 * noise sigma:
 *
 *   mu_n  = sum_m P[n - m] rho_m                          (Methods, Eqs. 1-2)
 *   L_n   = sum_{phi >= 0} Normal(w_n; G_n phi + o_n, sigma_n^2)
 *                          * Poisson(phi; mu_n)           (Eqs. 3-6)
 *   post  ~ prod_n L_n(mu_n) * prod_m p(rho_m)            (Eq. 9, separable prior)
 *
 * by Metropolis-within-Gibbs sweeps: pixels whose PSF footprints do not
 * overlap are conditionally independent (Methods, "Parallelization
 * Technique"), so each colour of a footprint colouring is updated in
 * parallel.  The posterior mean is the deconvolved image; the variance gives
 * the uncertainty (Results, "Uncertainty").
 *
 * Conventions shared by every entry point:
 *   - Images are row-major [height][width] float32; multi-chain arrays are
 *     [n_chains][height][width].  The object lattice is the pixel lattice and
 *     rho is zero outside the frame ("same"-size convolution).
 *   - on_device = 1: the pointer is HIP device memory readable from the
 *     context's stream; on_device = 0: host memory.  The library copies every
 *     input into buffers it owns; the caller owns (and frees) its buffers.
 *     Device inputs may be reused once the context's stream has passed the
 *     copy (the call returns after enqueueing it).
 *   - Work is enqueued on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return data to host memory synchronise that stream.
 *   - Every function returns a bdc_status; nothing aborts the process and no
 *     C++ exception crosses the boundary.  bdc_last_error() holds a message
 *     for the last failing call on that context.
 *   - A context is not thread-safe: use one context per host thread.
 *   - Call order: create -> set_psf -> set_camera_maps -> init -> sweep* ->
 *     posterior_moments / rhat / get_state.  Out-of-order calls return
 *     BDC_ESTATE.  set_psf or set_camera_maps after init invalidate the state
 *     (init must be called again).
 */
#ifndef BDC_H
#define BDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdc_ctx bdc_ctx;

typedef enum {
    BDC_OK = 0,
    BDC_EINVAL = -1,      /* bad shape, size or value */
    BDC_ENOMEM = -2,      /* device or host allocation failed */
    BDC_EDEVICE = -3,     /* a HIP call failed */
    BDC_ESTATE = -4,      /* call out of order */
    BDC_ENOTFINITE = -5   /* NaN or Inf in an input */
} bdc_status;

/* Scans (Methods, "Parallelization Technique"; all are systematic scans that
 * visit every pixel once per sweep with disjoint footprints inside a group):
 *   CHROMATIC     colour (y mod s, x mod s), one launch per colour;
 *   BLOCK         B x B blocks in four parity phases, the s*s colours inside a
 *                 block in order, each footprint term evaluated directly;
 *   BLOCK_SERIES  the same scan and groups as BLOCK with B in [s - 1, s] and
 *                 s <= 31; each footprint term comes from a cached local
 *                 series of the pixel's log-likelihood inside a radius where
 *                 its truncation error is provably below 1.5e-9 per term
 *                 (1.5e-6 over a 31 x 31 footprint), else directly;
 *   BLOCK9_SERIES the block-series terms over B x B blocks in nine phases
 *                 (block (by, bx) has phase (by mod 3) * 3 + bx mod 3, so
 *                 blocks of one phase lie three blocks apart) with B in
 *                 [(s - 1)/2, s] (default ceil((s - 1)/2)) and s <= 31: groups
 *                 phase * s * s + colour, 9 s * s of them, one wavefront per
 *                 block.
 * AUTO (block_size 0) picks, for a frame of at least 2 s rows and columns,
 * BLOCK9_SERIES for s <= 21 (B = s up to s = 11, else (s - 1)/2 rounded up),
 * BLOCK_SERIES for s <= 31 (B = s - 1), else BLOCK; CHROMATIC for smaller
 * frames.  With a nonzero block_size it picks BLOCK_SERIES when B fits it,
 * else BLOCK.  BLOCK_SERIES chosen explicitly with block_size 0 takes B = s - 1. */
enum { BDC_SCHED_AUTO = 0, BDC_SCHED_CHROMATIC = 1, BDC_SCHED_BLOCK = 2, BDC_SCHED_BLOCK_SERIES = 3,
       BDC_SCHED_BLOCK9_SERIES = 4 };
/* Priors (Methods, Prior; posterior of Eq. 9):
 *   FLAT       flat on (0, inf) per pixel;
 *   GAMMA      Gamma(prior_a, rate prior_b) per pixel;
 *   DIRICHLET  the Dirichlet-OTF prior of Eqs. 7-8 read per chunk: the object is
 *              cut into the B x B blocks of the block-phase scan (smaller at the
 *              bottom and right edges) and each chunk gets the Dirichlet of
 *              x_k = |F_k| / sum_j |F_j|, F its 2-D DFT over the chunk, with
 *              concentration alpha_k = |OTF_k| / sum_j |OTF_j|, the OTF being the
 *              DFT of the PSF wrapped onto the chunk's grid (centre at index 0),
 *              alpha floored at 1e-6 / K and renormalised; the whole spectrum
 *              (k and -k) enters.  Needs the block-phase scan (schedule AUTO or
 *              BLOCK) with block_size in [s - 1, s] (0 = s) and a PSF side s <= 31;
 *              the log-posterior trace includes every chunk's log prior.  Block
 *              moves (bdc_unet.h) and batches do not take this prior (EINVAL). */
enum { BDC_PRIOR_FLAT = 0, BDC_PRIOR_GAMMA = 1, BDC_PRIOR_DIRICHLET = 2 };
/* Cameras:
 *   SCMOS  w = G phi + o + Normal(0, sigma^2) per pixel (Methods, Eqs. 3-6);
 *   EMCCD  the electron-multiplication stage of the Discussion as an extra
 *          latent: photoelectrons phi ~ Poisson(mu), the register's output
 *          x ~ Gamma(phi, 1) in photon units for phi >= 1 (x = 0 for phi = 0),
 *          reading w = o + G x, read noise sigma on the zero-photon reading.
 *          With c = (w - o)/G the pixel factor is
 *            e^-mu [ Normal(w; o, sigma^2) + [c > 0] e^-c sqrt(mu/c) I_1(2 sqrt(mu c)) / G ]
 *          (I_1 the modified Bessel function), evaluated in closed form; it
 *          runs in the CHROMATIC and BLOCK scans (AUTO picks BLOCK, or
 *          CHROMATIC for small frames; the series scans refuse it, EINVAL),
 *          with every prior, with block moves and in batches. */
enum { BDC_CAMERA_SCMOS = 0, BDC_CAMERA_EMCCD = 1 };
/* Object lattice (Methods, Image Formation Model, Eqs. 1-2: the mean of pixel n
 * integrates the PSF-blurred object over the pixel).  object_sub = k > 1
 * discretises the object on k x k cells per camera pixel: rho is a
 * (k height) x (k width) array (row-major, cell (y, x) in pixel (y / k, x / k)),
 * the PSF passed to bdc_set_psf is sampled on that lattice (odd side s <= 63,
 * centred), and mu_n = sum over the k x k cells c of pixel n of (P (x) rho)_c,
 * zero outside the lattice.  The frame, the camera maps, bdc_get_mu and
 * bdc_loglik stay on the pixel lattice ([height][width]); everything about
 * rho (init's rho0, get/set_rho, moments, R-hat and MCSE maps, window mean,
 * samples, quantiles, CV map, debug records) is on the object lattice.  With
 * s_p = 2 floor((s/2 + k - 1)/k) + 1 the side of a cell's pixel footprint, the
 * scans are CHROMATIC (k^2 s_p^2 colours: cell phase (y mod k, x mod k) major,
 * then the pixel position mod s_p) and BLOCK (blocks of block_size pixels in
 * [s_p - 1, 4 s_p], 0 = max(s_p, min(4 s_p, 8)), four phases of k^2 s_p^2
 * groups each, the k^2 footprint tables and the block's region within 64 KiB
 * of LDS); AUTO picks BLOCK when the frame is at least 2 s_p pixels on each
 * side and it fits, else CHROMATIC; the series scans refuse it (EINVAL).  The
 * default start gives each cell max(c, 1/2)/k^2 exp(xi/2) of its pixel's
 * photon estimate c.  Flat and Gamma priors, both cameras; the Dirichlet-OTF
 * prior, batches, Richardson-Lucy, the learned start, block moves and training
 * targets take k = 1 only (EINVAL). */

typedef struct {
    int32_t  height, width;   /* frame = object lattice; each in [1, 32768], H*W <= 2^27 */
    int32_t  n_chains;        /* independent chains, in [1, 64]                      */
    int32_t  prior_kind;      /* BDC_PRIOR_FLAT, BDC_PRIOR_GAMMA or BDC_PRIOR_DIRICHLET */
    float    prior_a;         /* Gamma shape (> 0) when prior_kind = GAMMA           */
    float    prior_b;         /* Gamma rate (>= 0) when prior_kind = GAMMA           */
    int32_t  burn_in;         /* sweeps with step adaptation; moments start after    */
    float    log_step0;       /* initial log of the per-pixel log-normal walk step   */
    int32_t  schedule;        /* BDC_SCHED_*                                         */
    int32_t  block_size;      /* B for the block-phase scan (>= PSF side - 1), 0 = auto */
    int32_t  rhat_block;      /* sweeps per blocked-moment batch (R-hat, MCSE); 0 = 25 */
    int32_t  max_sweeps;      /* capacity of the blocked-moment store; 0 = 4096      */
    uint64_t seed;            /* Philox4x32-10 key (low word, high word)             */
    int32_t  camera;          /* BDC_CAMERA_SCMOS or BDC_CAMERA_EMCCD                */
    int32_t  object_sub;      /* object cells per pixel side k in [0, 4]; 0 or 1: object
                                 lattice = pixel lattice (see "Object lattice" above)  */
} bdc_config;

/* Fills *cfg with defaults: 1 chain, flat prior, burn_in 0, log_step0 -1.5,
 * automatic schedule, rhat_block 25, max_sweeps 4096, seed 0, sCMOS camera. */
void bdc_config_default(bdc_config* cfg);

/* Creates a context.  hip_stream is a hipStream_t (NULL = null stream).
 * Allocates the per-chain state in device memory (about 40 bytes per pixel
 * per chain plus the blocked-moment store).  EINVAL on a bad config. */
bdc_status bdc_create(const bdc_config* cfg, void* hip_stream, bdc_ctx** out);

/* Sets the shift-invariant PSF (Methods, "Image Formation Model": PSF(r - r'),
 * pixel-integrated, Eq. 1).  ph == pw, odd, at most 63; all entries finite and
 * >= 0 with a positive sum.  The library normalises it to sum 1.  The kernel
 * index [dy + r][dx + r] weights rho at offset (-dy, -dx) in mu (convolution). */
bdc_status bdc_set_psf(bdc_ctx* ctx, const float* psf, int32_t ph, int32_t pw, int32_t on_device);

/* Sets the camera calibration (Methods, Eq. 4): gain G (ADU per photon, > 0),
 * offset o (ADU, finite) and read-noise standard deviation sigma (ADU, > 0).
 * per_pixel = 1: each pointer is an [H][W] map; per_pixel = 0: each points to
 * one scalar, used for every pixel (the paper's fallback without maps). */
bdc_status bdc_set_camera_maps(bdc_ctx* ctx, const float* gain, const float* offset,
                               const float* read_sigma, int32_t per_pixel, int32_t on_device);

/* Uploads the raw frame w (ADU, [H][W], finite: the measurement of Methods,
 * Eq. 5) and initialises every chain of the sampler of Methods, Prior (the
 * posterior of Eq. 9).  rho0: NULL for the default start
 * rho_m = max(c_m, 1/2) exp(xi_m / 2), with c_m = (w_m - o_m) / G_m the photon
 * estimate and xi from Philox stream 2 (overdispersed per chain); otherwise
 * [n_chains][H][W] strictly positive values.  Resets the sweep counter, the
 * moments and the acceptance counters.  EINVAL on a NULL frame, ENOTFINITE on
 * a non-finite frame or camera value, EINVAL on a non-positive gain or read
 * noise or a rho0 entry that is not finite and > 0; ESTATE before set_psf and
 * set_camera_maps.  Synchronises. */
bdc_status bdc_init(bdc_ctx* ctx, const float* image_adu, const float* rho0, int32_t on_device);

/* Enqueues n >= 0 full sweeps and returns without waiting.  One sweep of the
 * Gibbs-style scan of Methods, Parallelization Technique (pixels whose PSF
 * footprints are disjoint updated together, each update conditioned on every
 * earlier one): mu = P (x) rho from scratch (Eqs. 1-2); every colour (or block
 * phase) in order, each pixel proposing rho' = rho exp(step * xi) and
 * accepting iff log u < Delta log posterior + log(rho'/rho), the posterior of
 * Eq. 9 with the likelihood of Eqs. 3-6; step adaptation while the sweep index
 * is below burn_in; moments and the log-posterior trace after.  ESTATE before
 * bdc_init; EINVAL for n < 0; a failed launch is reported as EDEVICE by this
 * call or the next synchronising one.  Sweeps beyond max_sweeps still run, but
 * the blocked diagnostics (R-hat, MCSE, window mean) then return ESTATE. */
bdc_status bdc_sweep(bdc_ctx* ctx, int32_t n);

/* Posterior mean and variance of rho over the post-burn-in sweeps
 * (Results, "Uncertainty": the mean is the deconvolved image).  chain >= 0:
 * that chain (variance M2 / (n - 1)); chain = -1: all chains pooled (sample
 * mean and variance of the n_chains * n draws).  mean/var: [H][W], either
 * may be NULL.  *n_samples receives n per chain.  ESTATE if n < 2.
 * Synchronises the stream. */
bdc_status bdc_posterior_moments(bdc_ctx* ctx, int32_t chain, float* mean, float* var,
                                 int64_t* n_samples, int32_t on_device);

/* Split R-hat (Gelman et al., BDA3 sec. 11.4) over the second half of the
 * sweeps run so far, in whole rhat_block batches: per pixel on log rho (its
 * 99th percentile over pixels, the upper edge of its bin in a device
 * histogram with 1e-5 bins below 1.5 and 1e-3 bins up to 11.5; INFINITY
 * beyond), and on the per-chain log-posterior trace.  Needs n_chains >= 2
 * and at least 4 completed batches; otherwise ESTATE.  Synchronises. */
bdc_status bdc_rhat(bdc_ctx* ctx, float* rhat_p99, float* rhat_logpost);

/* Per-pixel split R-hat map ([H][W]) as used by bdc_rhat. */
bdc_status bdc_rhat_map(bdc_ctx* ctx, float* rhat, int32_t on_device);

/* Posterior mean of rho over the draws of bdc_rhat's window (the second half
 * of the completed batches, all chains pooled): the estimate at the moment
 * the convergence criterion is evaluated (Methods, Prior: the estimator is
 * the mean of decorrelated samples after convergence).  [H][W]; needs at
 * least 4 completed batches; synchronises. */
bdc_status bdc_window_mean(bdc_ctx* ctx, float* mean, int32_t on_device);

/* Batch windows of the diagnostics after t sweeps under cfg (host arithmetic
 * only; no device work, usable without a GPU).  A batch counts once all of its
 * rhat_block sweeps have run and lie inside the max_sweeps store.  With `done`
 * such batches: R-hat and the window mean use batches [b_lo, b_lo + 2 half),
 * half = done / 4, b_lo = done - 2 half (the second half of the completed
 * batches, whose log-posterior trace entries [b_lo, b_lo + 2 half) * rhat_block
 * all lie below max_sweeps); MCSE uses the post-burn-in batches [b0, b0 + nb),
 * b0 = ceil(burn_in / rhat_block).  Zero rhat_block / max_sweeps mean the
 * defaults (25, 4096).  ESTATE when t > max_sweeps (bdc_rhat, bdc_rhat_map,
 * bdc_window_mean and bdc_mcse then return ESTATE too: their windows would need
 * sweeps the store does not hold); EINVAL for a NULL or negative config.
 * Any output pointer may be NULL. */
bdc_status bdc_diag_window(const bdc_config* cfg, int64_t t, int32_t* b_lo, int32_t* half, int32_t* b0,
                           int32_t* nb);

/* Batch-means Monte Carlo standard error of the posterior mean per pixel,
 * pooled over chains ([H][W]), using the post-burn-in rhat_block batches
 * (needs >= 2 of them).  Synchronises. */
bdc_status bdc_mcse(bdc_ctx* ctx, float* mcse, int32_t on_device);

/* Current state: rho and the per-pixel log step, [n_chains][H][W] each (either
 * may be NULL); *sweep receives the index of the next sweep.  Synchronises. */
bdc_status bdc_get_rho(bdc_ctx* ctx, float* rho, float* log_step, int64_t* sweep, int32_t on_device);

/* Expected image mu = P (x) rho of the current state, recomputed from rho
 * ([n_chains][H][W]).  Synchronises. */
bdc_status bdc_get_mu(bdc_ctx* ctx, float* mu, int32_t on_device);

/* Per-pixel log-likelihood log L_n(mu_n) (Eq. 6 factor, including the
 * -log(sqrt(2 pi) sigma_n) normalisation) at mu = P (x) rho of chain `chain`,
 * [H][W].  Synchronises. */
bdc_status bdc_loglik(bdc_ctx* ctx, int32_t chain, float* ell, int32_t on_device);

/* Log-posterior trace: one value per chain per completed sweep since init,
 * [sweeps][n_chains] doubles; *count receives the number of sweeps stored
 * (capacity max_sweeps).  trace may be NULL to query the count. */
bdc_status bdc_logpost_trace(bdc_ctx* ctx, double* trace, int64_t capacity, int64_t* count);

/* Accepted and proposed updates per chain since init (int64 [n_chains] each). */
bdc_status bdc_accept_stats(bdc_ctx* ctx, int64_t* accepted, int64_t* proposed);

/* Checkpoint.  bdc_get_state with buf = NULL stores the needed size in *bytes;
 * otherwise writes the whole sampler state (rho, log steps, sweep index,
 * moments, blocked moments, trace, counters) into buf (host memory).
 * bdc_set_state restores a buffer written by a context with the same config,
 * PSF and camera, after init.  Resuming is bit-exact: the random numbers are a
 * function of (pixel, sweep, chain) only.  Both synchronise. */
bdc_status bdc_get_state(bdc_ctx* ctx, void* buf, size_t* bytes);
bdc_status bdc_set_state(bdc_ctx* ctx, const void* buf, size_t bytes);

/* Overwrites rho and the log steps of every chain ([n_chains][H][W], rho > 0)
 * and the sweep index; moments are left as they are.  For tests that start
 * the GPU and the CPU oracle from one shared state. */
bdc_status bdc_set_rho(bdc_ctx* ctx, const float* rho, const float* log_step, int64_t sweep,
                       int32_t on_device);

/* Parity hook: recomputes mu from rho, then runs schedule groups [g0, g1) of
 * the current sweep (groups are the colours 0..s*s-1 of the pixel-chromatic
 * scan, or phase*s*s + colour of the block-phase scan), exactly as bdc_sweep
 * would, without moments and without advancing the sweep index.  For every
 * updated pixel writes Delta (the log acceptance ratio) and the decision into
 * [n_chains][H][W] arrays (other entries untouched; either may be NULL).
 * Synchronises. */
bdc_status bdc_debug_run_groups(bdc_ctx* ctx, int32_t g0, int32_t g1, float* delta,
                                uint8_t* accepted, int32_t on_device);

/* Number of schedule groups of the configured scan, and the scan in use
 * (BDC_SCHED_CHROMATIC, BDC_SCHED_BLOCK or BDC_SCHED_BLOCK_SERIES) with its
 * block side. */
bdc_status bdc_schedule_info(bdc_ctx* ctx, int32_t* n_groups, int32_t* schedule, int32_t* block);

/* Philox4x32-10 on the device (Salmon et al., SC'11): n counters of 4 words
 * ([n][4] uint32) under key (key0, key1) -> [n][4] outputs.  Device pointers.
 * Synchronises.  Exposed so the generator can be checked bit for bit. */
bdc_status bdc_philox(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* out,
                      void* hip_stream);

/* Measurement.  enable = 1: later bdc_sweep calls launch kernel by kernel
 * (no graph replay) and record HIP events on the library's own stream, the
 * stream the kernels run on, after the forward/proposal kernel, after every
 * colour or phase pass and after the moments kernels.  enable = 0 turns it off
 * and drops pending marks.  Synchronises. */
bdc_status bdc_profile(bdc_ctx* ctx, int32_t enable);

/* Reads and resets the measurement since the last read: ms[3] accumulated
 * kernel milliseconds and launches[3] launch counts for the classes
 * (0 forward/proposal, 1 colour or phase passes, 2 moments); work[6] = phi-sum
 * terms of direct footprint evaluations, footprint likelihood evaluations,
 * and for the block-series scan: the footprint terms evaluated directly, the
 * series anchored from scratch (new ring rows), the phi-sum terms of those,
 * and the series re-anchored inside a direct evaluation (counted on every
 * sweep, profiled or not).  Any pointer may be NULL.  Synchronises. */
bdc_status bdc_profile_read(bdc_ctx* ctx, double* ms, int64_t* launches, int64_t* work);

/* Autotuner of the scan: for each candidate block side blocks[i] (0 = the
 * pixel-chromatic scan; b > 0 the block-phase scan with B = b, skipped when
 * outside [psf side - 1, 4 * psf side] or above 64 KiB of LDS; -1000 < b < 0
 * the block-series scan with B = -b, b <= -1000 the nine-phase block-series
 * scan with B = -b - 1000, each skipped when it does not fit or the context
 * reads an EMCCD camera),
 * times `sweeps` real sweeps with HIP events on the library's stream and
 * stores the mean milliseconds per sweep in ms_per_sweep[i] (INFINITY when
 * skipped).  The fastest candidate becomes the context's scan; *best receives
 * it (INT32_MIN when every candidate was skipped).  The timed sweeps advance the chain like bdc_sweep, so call this during
 * burn-in.  Synchronises. */
bdc_status bdc_autotune(bdc_ctx* ctx, const int32_t* blocks, int32_t n, int32_t sweeps, float* ms_per_sweep,
                        int32_t* best);

/* Selects the scan without timing (e.g. a cached autotuner result): schedule
 * BDC_SCHED_* and block side (0 = automatic), validated like bdc_create's
 * config.  Allowed at any point after set_psf; a batch holding this context
 * must be recreated. */
bdc_status bdc_set_schedule(bdc_ctx* ctx, int32_t schedule, int32_t block);

/* Batched sweeps.  A batch fuses the sweeps of several initialised contexts
 * ("tiles": frames of different sizes, PSFs and cameras, each with its own
 * chains and seeds) into one HIP graph per sweep of levels (forward/proposal
 * tiles, the block phases: four, or nine for nine-phase tiles, moments chunks,
 * trace), each non-empty level one launch per kind of work (block-series,
 * nine-phase block-series, sCMOS block-phase and EMCCD block-phase tiles apart) that
 * runs every work item of that kind for all tiles and chains at once, longest
 * first; launch boundaries order the levels, so no workgroup waits on another.  Results are those of
 * calling bdc_sweep on each tile: every tile keeps its own state, moments and
 * parity hooks, read through its own context.  Tiles must use a block-phase or
 * block-series scan (EMCCD tiles: block-phase only, as their contexts) and a
 * separable prior on the pixel lattice (EINVAL otherwise), live on one device and outlive the batch; changing a tile's PSF or
 * camera invalidates the batch (bdc_batch_sweep then returns ESTATE). */
typedef struct bdc_batch bdc_batch;
bdc_status bdc_batch_create(bdc_ctx* const* tiles, int32_t n_tiles, void* hip_stream, bdc_batch** out);

/* Enqueues n sweeps of every tile (async), ordered after the caller's stream
 * and each tile's earlier work; later calls on a tile are ordered after it. */
bdc_status bdc_batch_sweep(bdc_batch* b, int32_t n);

/* Synchronises the batch's stream; BDC_EDEVICE if a launch failed. */
bdc_status bdc_batch_check(bdc_batch* b);

/* Work items per sweep, the largest launch's workgroup count and the largest
 * LDS bytes per workgroup among the launches. */
bdc_status bdc_batch_info(bdc_batch* b, int64_t* n_items, int32_t* grid, int32_t* lds_bytes);
const char* bdc_batch_last_error(const bdc_batch* b);
void bdc_batch_destroy(bdc_batch* b);

/* ---- Richardson-Lucy, the paper's baseline (Introduction; Results,
 * Simulated Data) ----
 * n_iter iterations of rho <- rho * (P^T (d / (P rho))) / (P^T 1) (Richardson
 * 1972; Lucy 1974) on the context's frame: d = max((w - o) / G, 0), P the
 * normalised PSF with the same-size zero-padded convolution of the sampler,
 * P^T the correlation, rho_0 = mean(d) everywhere, sums in FP64, state in
 * FP32; a pixel with P rho = 0 contributes nothing.  out: [H][W].  Needs init;
 * uses the context's scratch buffers (no effect on the chains).  Synchronises. */
bdc_status bdc_richardson_lucy(bdc_ctx* ctx, int32_t n_iter, float* out, int32_t on_device);

/* Richardson-Lucy warm start (after bdc_init): every chain restarts at
 * rho = max(rl, 1e-3) exp(xi / 2), rl the estimate after n_iter iterations and
 * xi from Philox stream 2 at sweep 0 (one draw per chain: overdispersed
 * starts, as R-hat requires); log steps = log_step0.  Resets the sweep counter,
 * moments and acceptance counters as bdc_init does. */
bdc_status bdc_init_rl(bdc_ctx* ctx, int32_t n_iter);

/* ---- Posterior samples, quantiles, CV (Results, "Our package": the sampler
 * returns many candidate deconvolved images; "Uncertainty": quantiles,
 * variance and the coefficient of variation CV = std / mean per pixel) ---- */

/* Thinned export: from then on, every post-burn-in sweep t with
 * (t - burn_in) % thin == 0 stores every chain's rho into slot
 * (t - burn_in) / thin of a device stack [capacity][n_chains][H][W] owned by the
 * context (the first `capacity` such sweeps; later ones are not stored).
 * thin = 0 or capacity = 0 turns the export off and frees the stack (allowed
 * at any time).  Turning it on is allowed before init or while the sweep index
 * is <= burn_in (else ESTATE).  ENOMEM if the stack does not fit. */
bdc_status bdc_set_export(bdc_ctx* ctx, int32_t thin, int32_t capacity);

/* Stored samples [first, first + count) into out ([count][n_chains][H][W]);
 * *n_stored (may be NULL) receives the number stored so far.  out = NULL or
 * count = 0 only queries the count.  EINVAL for a range beyond the stored
 * samples.  Synchronises. */
bdc_status bdc_samples(bdc_ctx* ctx, float* out, int64_t first, int64_t count, int64_t* n_stored,
                       int32_t on_device);

/* Per-pixel quantiles of all stored samples of all chains (n = stored x
 * n_chains values per pixel, 1 <= n <= 4096): probs (host, n_probs levels in
 * [0, 1]) -> out [n_probs][H][W].  With the sorted values x_0 <= ... <= x_{n-1}
 * and h = (n - 1) p, q = x_floor(h) + (h - floor(h)) (x_floor(h)+1 - x_floor(h))
 * (linear interpolation between order statistics; an order statistic itself
 * when h is an integer).  ESTATE without stored samples.  Synchronises. */
bdc_status bdc_quantiles(bdc_ctx* ctx, const float* probs, int32_t n_probs, float* out, int32_t on_device);

/* The same quantiles of caller data: samples [n][n_pix] (device), probs
 * [n_probs] (device), out [n_probs][n_pix] (device), on hip_stream (NULL =
 * null stream); 1 <= n <= 4096.  Synchronises the stream. */
bdc_status bdc_quantiles_of(const float* samples, int64_t n, int64_t n_pix, const float* probs, int32_t n_probs,
                            float* out, void* hip_stream);

/* Coefficient of variation sqrt(var) / mean per pixel of the pooled posterior
 * moments (as bdc_posterior_moments with chain = -1), [H][W].  ESTATE before 2
 * post-burn-in sweeps.  Synchronises. */
bdc_status bdc_cv_map(bdc_ctx* ctx, float* cv, int32_t on_device);

/* Message of the last failing call on ctx (or of the last failing
 * bdc_create / bdc_philox when ctx is NULL).  Never NULL. */
const char* bdc_last_error(const bdc_ctx* ctx);

/* Frees the context and its device memory (synchronises its stream first). */
void bdc_destroy(bdc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BDC_H */
