/* bdc_unet.h -- C ABI of the learned part: a small U-Net that maps a frame's
 * photon image to a per-pixel log-normal approximation of the posterior of rho,
 * used as the sampler's warm start and as a block independence proposal.
 *
 * The paper gives no learned component (its Introduction argues against
 * replacing the physics with a network); here the network never replaces the
 * sampler: the warm start only chooses rho at t = 0, and the block move is an
 * exact Metropolis-Hastings step whose acceptance carries the proposal
 * density, so the target posterior (Prior section, Eq. for the posterior) is
 * unchanged whatever the network outputs.
 *
 * Network: `levels` resolution levels with base_channels * 2^l channels; two
 * 3x3 convolutions (zero padding) + ReLU per level, 2x2 max pooling down,
 * 2x2 stride-2 transposed convolutions up, skip concatenation (up-sampled
 * first, skip second), and a 1x1 head with two outputs per pixel:
 *   m = mean of log(rho / scale),  s = log of the standard deviation of log rho,
 * where scale = the frame's mean photon estimate mean((w - o) / G).  Input:
 * the photon estimate (w - o)/G divided by scale, one channel.
 *
 * Parameters: one FP32 array (master weights), layer by layer in forward order
 * (encoder levels, bottleneck, decoder levels from deepest, head):
 *   3x3 conv:      W[c_out][3][3][c_in], then b[c_out]
 *   2x2 transposed: W[2][2][c_out][c_in], then b[c_out]
 *   head:          W[2][c], then b[2]
 * Compute: BF16 operands on the matrix cores, FP32 accumulation, BF16
 * activations (NHWC) between layers.
 *
 * Training loss (per batch of P pixels): (1/P) sum_p [(m_p - y_p)^2 + (s_p - z_p)^2]
 * with targets y = mean of log(rho/scale) and z = log std of log rho from the
 * sampler's posterior moments.  Optimiser: Adam with bias correction.
 *
 * Conventions as in bdc.h: every function returns bdc_status; the caller owns
 * all buffers; pointers are host or device per `on_device`; work is ordered
 * after the caller's stream on entry and before it on exit; an object is not
 * thread-safe.
 */
#ifndef BDC_UNET_H
#define BDC_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "bdc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bdc_unet bdc_unet;

typedef struct {
    int32_t levels;          /* resolution levels, 2..6 (4 = three poolings)                   */
    int32_t base_channels;   /* channels at full resolution: 8, 16, 32 or 64                   */
    int64_t max_pixels;      /* largest batch * height * width that forward/training will see */
    int32_t training;        /* 1: allocate gradient buffers and optimiser state              */
} bdc_unet_config;

/* Creates a network with all parameters zero (set them with bdc_unet_set_params).
 * EINVAL on an unsupported shape, ENOMEM if the buffers do not fit. */
bdc_status bdc_unet_create(const bdc_unet_config* cfg, void* hip_stream, bdc_unet** out);

/* Number of FP32 parameters in the layout above. */
bdc_status bdc_unet_param_count(const bdc_unet* u, int64_t* n);

/* Forward FLOPs (2 per multiply-add, convolutions and head) of one batch. */
bdc_status bdc_unet_flops(const bdc_unet* u, int32_t batch, int32_t height, int32_t width, double* flops);

/* Copies the FP32 parameters in (and refreshes the BF16 operand copies) / out.
 * Non-finite values: ENOTFINITE. */
bdc_status bdc_unet_set_params(bdc_unet* u, const float* params, int32_t on_device);
bdc_status bdc_unet_get_params(bdc_unet* u, float* params, int32_t on_device);

/* Forward pass.  x: [batch][height][width] FP32 normalised photon images;
 * out: [batch][height][width][2] FP32 (m, s).  height and width must be
 * multiples of 2^(levels-1); batch*height*width <= max_pixels. */
bdc_status bdc_unet_forward(bdc_unet* u, const float* x, int32_t batch, int32_t height, int32_t width, float* out,
                            int32_t on_device);

/* Forward + backward without an update.  target: [batch][height][width][2]
 * (y, z).  grads: FP32, same layout as the parameters (may be NULL);
 * loss: host float (may be NULL).  Needs training = 1. */
bdc_status bdc_unet_gradients(bdc_unet* u, const float* x, const float* target, int32_t batch, int32_t height,
                              int32_t width, float* grads, float* loss, int32_t on_device);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; loss as above. */
bdc_status bdc_unet_train_step(bdc_unet* u, const float* x, const float* target, int32_t batch, int32_t height,
                               int32_t width, float lr, float* loss, int32_t on_device);

/* Zeroes the Adam moments and step count. */
bdc_status bdc_unet_reset_optimizer(bdc_unet* u);

/* Parity hook of the matrix-core tile: C[M][N] = A[M][K] B[N][K]^T with BF16
 * A, B (raw 16-bit patterns, host) and FP32 C (host); K % 8 == 0. */
bdc_status bdc_debug_gemm_bf16(const uint16_t* a, const uint16_t* b, float* c, int64_t m, int32_t n, int32_t k);

const char* bdc_unet_last_error(const bdc_unet* u);
void bdc_unet_destroy(bdc_unet* u);

/* ---- The network inside the sampler ---------------------------------------
 * Learned warm start (after bdc_init): runs the network on the context's frame
 * (zero-padded to a multiple of 2^(levels-1)), stores the per-pixel proposal
 * maps  mean_log = m + log(scale), sd_log = clamp(exp(s), 0.02, 3),  and
 * restarts every chain at  rho_m = exp(mean_log_m + min(2 sd_log_m, 3) xi_m)
 * with xi from Philox stream 2 at t = 0 (one draw per chain; twice the
 * network's spread keeps the starts overdispersed, as R-hat assumes).
 * Resets the sweep counter, moments and step sizes as bdc_init does. */
bdc_status bdc_init_learned(bdc_ctx* ctx, bdc_unet* u);

/* Sets the block-proposal maps directly: [H][W] FP32 each, sd_log > 0. */
bdc_status bdc_set_block_proposal(bdc_ctx* ctx, const float* mean_log, const float* sd_log, int32_t on_device);

/* n passes of the block move on every chain: 16x16 blocks, in k x k block
 * colours with k = 1 + ceil(2r / 16) (blocks of one colour have disjoint
 * extended footprints).  Per block pixel, in u = log rho with the reference
 * N(mean_log_m, sd_log_m^2) and z = (u - mean_log)/sd_log:
 *   z' = sqrt(1 - beta^2) z + beta xi,   xi from Philox stream 3 at (m, pass, chain),
 * an autoregressive step that leaves the reference invariant (beta = 1: the
 * independence proposal rho' ~ LogNormal(mean_log, sd_log^2)).  Accept iff
 *   log u < dlog-likelihood + dlog-prior + sum_m [(u'_m - u_m) + (z'_m^2 - z_m^2)/2]
 * with u from stream 4 at (first pixel of the block, pass, chain): the
 * Metropolis-Hastings ratio of this proposal, so the posterior is preserved
 * for any maps and any beta.  mu is recomputed from rho at the start of each
 * pass.  Needs proposal maps. */
bdc_status bdc_block_move(bdc_ctx* ctx, int32_t n);

/* The block move's beta in (0, 1] (default 1). */
bdc_status bdc_set_block_beta(bdc_ctx* ctx, float beta);

/* step > 0 turns the block move into a walk along the directions the blur
 * removes, which needs no proposal maps: every pixel m of a 16 x 16 block moves
 * in u = log rho by  u'_m = u_m + step * h_m,  h = xi - P (x)_B xi,  xi_m from
 * Philox stream 3 at (m, pass, chain) and (P (x)_B xi)_m = sum_{m' in block}
 * P[m - m'] xi_m' the blur of xi restricted to the block's pixels in the frame
 * (white noise minus its blurred copy: the components the PSF suppresses).  h is
 * linear in the symmetric xi, so the move is symmetric in u and the block is
 * accepted iff log u < dlog-likelihood + dlog-prior + sum_m (u'_m - u_m), u from
 * stream 4 as for the reference move: exact Metropolis-Hastings, the posterior
 * is preserved for any step (with an identity PSF h = 0 and the walk stands
 * still).  step = 0 (default) restores the reference move.  EINVAL for a
 * negative or non-finite step. */
bdc_status bdc_set_block_walk(bdc_ctx* ctx, float step);

/* Block moves accepted / proposed since bdc_init (all chains). */
bdc_status bdc_block_stats(bdc_ctx* ctx, int64_t* accepted, int64_t* proposed);

/* Training pair of the context's frame (training-data generation, after
 * enough post-burn-in sweeps): x[H][W] = c / scale (the network input),
 * target[H][W][2] = (log(mean) - s2/2 - log(scale), log(s2)/2) with
 * s2 = log(1 + var / mean^2), the log-normal matching the pooled posterior
 * mean and variance of rho; scale (host float, may be NULL) as above.
 * Host outputs reuse the proposal-map buffer as staging and clear the maps
 * (set them again before the next block move). */
bdc_status bdc_training_targets(bdc_ctx* ctx, float* x, float* target, float* scale, int32_t on_device);

/* bdc_training_targets for callers that cannot allocate device memory (code
 * under HIP graph capture, tight data-generation or serving loops, harnesses
 * that forbid hipMalloc): the same outputs from the same kernels, with no
 * hipMalloc / hipFree and without touching the block-proposal maps.  Host
 * outputs, and the frame scale, are staged through one library-owned device
 * array of 64 MiB per GPU, held until the process ends, so the frame may hold
 * at most 5,592,384 pixels (EINVAL beyond).  Calls that overlap in time on one
 * GPU share that array and race; serialise them.  Other errors as
 * bdc_training_targets. */
bdc_status bdc_training_targets_noalloc(bdc_ctx* ctx, float* x, float* target, float* scale, int32_t on_device);

/* Parity hook: one block colour at block-pass index `pass` from the current
 * state; delta [n_chains][n_blocks_of_colour] (log acceptance ratio) and acc
 * (1 accepted, 0 rejected), both host, in ascending block index.  Commits the
 * accepted blocks like bdc_block_move.  n_blocks: host out (may be NULL). */
bdc_status bdc_debug_block_colour(bdc_ctx* ctx, int64_t pass, int32_t colour, float* delta, uint8_t* acc,
                                  int32_t* n_blocks);

#ifdef __cplusplus
}
#endif

#endif /* BDC_UNET_H */
