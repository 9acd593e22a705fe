// bdc_kernels.h -- host-side view of the gfx950 kernels (parameter blocks and
// launchers).  Everything here is plain C++ over device pointers; the kernels
// themselves live in bdc_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdc_consts.h"

namespace bdc {

struct Frame {                     // one frame (or one tile of a batch)
    int H, W, s, r;                // object lattice size, footprint side and radius
    int64_t N;                     // H * W: object cells (rho, its moments and draws)
    int C;                         // chains
    const float* psf;              // [s*s], sums to 1
    const uint16_t* psf_order;     // [s*s] footprint offsets by descending PSF weight
    const float4* pc;              // per pixel: (c, 2a, L0, iB), see PixConst
    const float* w;                // raw frame (ADU)
    const float* gain;             // camera maps (per pixel) or 1-element scalars
    const float* offset;
    const float* sigma;
    int cam_per_pixel;
    int camera = 0;                // 0: sCMOS reading, 1: EMCCD reading (pc holds (c, -1, log A, -c - log G))
    // Pixel lattice.  sub = 1: the object lattice (H = Hp, W = Wp).  sub = k > 1:
    // k x k object cells per pixel; pc, w, the camera maps and mu are [Hp][Wp],
    // psf holds k^2 pixel-footprint tables [phase][s][s] (phase = (y mod k) k +
    // x mod k of the cell): the light of a cell in pixel p reaching pixel p + d.
    int sub = 1;
    int Hp = 0, Wp = 0;
    int64_t Np = 0;
    uint2 key;                     // Philox key
    // Dirichlet-OTF prior per chunk (nullptr dir_am1: separable prior).  The
    // chunks are the B x B blocks of the block-phase scan (edge chunks smaller).
    const float* dir_am1 = nullptr;  // alpha_k - 1 per chunk shape: [4][B*B], shape = 2 (bottom edge) + (right edge)
    const double* dir_const = nullptr;  // [4]: lgamma(sum alpha) - sum_k lgamma(alpha_k) per shape
    double2* dir_F = nullptr;      // [C][H][W]: each chunk's spectrum F_k stored at the chunk's pixel (ky, kx)
    int dir_B = 0;                 // chunk side
};

constexpr int NCOUNTERS = 6;       // work counters of a context (State::counters)

struct State {
    float* rho;                    // [C][N]
    float* log_step;               // [C][N]
    float* mu;                     // [C][N]
    float* prop_rho;               // proposals of the current sweep, [C][N]
    float* prop_hast;              // log q-ratio + log prior ratio, [C][N]
    float* prop_logu;              // log of the accept uniform, [C][N]
    int64_t* t;                    // device copy of the sweep index
    unsigned long long* accepts;   // [C]
    unsigned long long* counters;  // [0] phi terms summed, [1] footprint evaluations,
                                   // [2] direct evaluations, [3] series anchored from scratch,
                                   // [4] their phi terms, [5] series re-anchored in a direct
                                   // evaluation (block-series scan)
};

struct Prior { int kind; float a, b; };

struct MomentBufs {
    float* mean;                   // Welford over post-burn-in sweeps, [C][N]
    float* m2;
    float* batch;                  // [n_batches][3][C][N]: mean rho, mean log rho, M2 log rho
    int rhat_block;
    int max_batches;
    double* lp_partial;            // [n_wg][C]
    double* trace;                 // [max_sweeps][C]
    int max_sweeps;
    double* dir_part = nullptr;    // [n_chunks][C]: log prior of each chunk (Dirichlet-OTF prior), or nullptr
    int n_chunks = 0;
};

hipError_t launch_pixel_consts(const Frame& f, float4* pc, int* bad, hipStream_t st);
hipError_t launch_init_state(const Frame& f, const State& S, const float* rho0, float log_step0, int* bad,
                             hipStream_t st);
size_t block_phase_lds(int B, int s);
size_t block_phase_sub_lds(int B, int s, int k);   // finer object lattice: k^2 footprint tables
hipError_t launch_forward_propose(const Frame& f, const State& S, const Prior& pr, int propose,
                                  hipStream_t st);
hipError_t launch_colour_pass(const Frame& f, const State& S, int burn_in, const double* inv_tab,
                              int colour, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st);
hipError_t launch_block_phase(const Frame& f, const State& S, int burn_in, const double* inv_tab,
                              int B, int phase, int k0, int k1, float* dbg_delta, uint8_t* dbg_acc,
                              hipStream_t st);
// Block-series scan (one active pixel per colour and block: B in [s - 1, s],
// s * s <= 4 * WG); needs block_series_lds(B, s) bytes of LDS per workgroup.
constexpr size_t BLOCK_SERIES_LDS_MAX = 80 * 1024;
size_t block_series_lds(int B, int s);
bool block_series_fits(int B, int s);
hipError_t launch_block_series(const Frame& f, const State& S, int burn_in, const double* inv_tab, int B,
                               int phase, int k0, int k1, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st);
// Block-series scan in nine phases (blocks of one phase three blocks apart: B in
// [(s - 1)/2, s], s * s <= 1024), one wavefront per block; phase in [0, 9).
size_t wave_series_lds(int B, int s);
bool wave_series_fits(int B, int s);
hipError_t launch_wave_series(const Frame& f, const State& S, int burn_in, int B, int phase, int k0, int k1,
                              float* dbg_delta, uint8_t* dbg_acc, hipStream_t st);
hipError_t launch_moments(const Frame& f, const State& S, const Prior& pr, const MomentBufs& M,
                          int burn_in, int advance, hipStream_t st);
// Dirichlet-OTF prior per chunk: every chunk's spectrum of rho into f.dir_F
// (before the block passes of a sweep), or every chunk's log prior into
// M.dir_part (for the log-posterior trace).
hipError_t launch_chunk_spectra(const Frame& f, const State& S, hipStream_t st);
hipError_t launch_chunk_logprior(const Frame& f, const State& S, const MomentBufs& M, hipStream_t st);
int chunk_count(const Frame& f);
hipError_t launch_loglik(const Frame& f, const float* mu, double* out, hipStream_t st);
hipError_t launch_rhat_map(const Frame& f, const MomentBufs& M, int b_lo, int half, float* rhat,
                           hipStream_t st);
hipError_t launch_hist(const float* v, int64_t n, float lo, float w_fine, int n_fine, float w_coarse, int n_coarse,
                       unsigned int* hist, hipStream_t st);
hipError_t launch_mcse(const Frame& f, const MomentBufs& M, int b0, int nb, float* mcse, hipStream_t st);
hipError_t launch_pooled_moments(const Frame& f, const MomentBufs& M, int64_t n, int chain,
                                 float* mean, float* var, hipStream_t st);
hipError_t launch_philox(const uint32_t* ctr, int64_t n, uint2 key, uint32_t* out, hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);

// Posterior samples (bdc_samples.hip): thinned export of rho into a device
// stack [slot][C][N], per-pixel quantiles (n <= QMAX values each), CV map.
constexpr int64_t QMAX = 4096;
hipError_t launch_export(const Frame& f, const float* rho, const int64_t* tp, int burn_in, int thin, int cap,
                         float* stack, hipStream_t st);
size_t quantile_lds(int64_t n);
hipError_t launch_quantiles(const float* v, int64_t n, int64_t stride, int64_t n_pix, const float* probs, int n_probs,
                            float* out, hipStream_t st);
hipError_t launch_cv(const float* mean, const float* var, int64_t n, float* cv, hipStream_t st);

// Richardson-Lucy (bdc_rl.hip): n_iter iterations on the frame's photon image
// into rho [N] (scratch q, norm [N] floats, part [ceil(N / WG)] doubles), and
// the warm start of every chain from an RL estimate.
hipError_t launch_richardson_lucy(const Frame& f, int n_iter, float* rho, float* q, float* norm, double* part,
                                  hipStream_t st);
hipError_t launch_rl_init(const Frame& f, const State& S, const float* rl, float floor_v, float log_step0,
                          hipStream_t st);

// Learned part (see bdc_unet.h): frame scale, network input, warm start, block move.
int block_period(int r);
int block_colour_count(const Frame& f, int colour);
size_t block_colour_lds(int s);
hipError_t launch_block_colour(const Frame& f, const State& S, const Prior& pr, const float* pm, const float* ps,
                               const double* inv_tab, int colour, uint32_t pass, float beta, float walk,
                               unsigned long long* bacc, float* dbg_delta, uint8_t* dbg_acc, hipStream_t st);
hipError_t launch_frame_scale(const Frame& f, double* part, float* scale, hipStream_t st);
hipError_t launch_window_mean(const Frame& f, const MomentBufs& M, int b0, int nb, float* out, hipStream_t st);
hipError_t launch_training_targets(const Frame& f, const float* mean, const float* var, const float* scale, float* x,
                                   float* tgt, hipStream_t st);
hipError_t launch_learned_input(const Frame& f, const float* scale, int Hp, int Wp, float* x, hipStream_t st);
hipError_t launch_learned_init(const Frame& f, const State& S, const float* out, int Wp, const float* scale,
                               float log_step0, float* pm, float* ps, hipStream_t st);

}  // namespace bdc

namespace bdc {

// ---------------------------------------------------------------------------
// Batched sweep: many frames (tiles) of different sizes and PSFs advance one
// sweep together.  Work items are (tile, chain, level, index); levels:
// 0 forward/proposal tiles, 1..9 block phases (four-phase tiles use 1..4),
// 10 moments chunks, 11 trace finalisation.  One launch per non-empty level
// and kind of work (a block-phase level
// launches its block-series tiles and its block-phase tiles separately) runs
// every item of that segment, longest first; launch boundaries are the only
// dependencies.  Each kind has its own kernel, so each gets the registers and
// LDS of its own body.
// ---------------------------------------------------------------------------
constexpr int NLEV = 12;
constexpr int LEV_MOMENTS = 10, LEV_FINALIZE = 11;
constexpr int FT_SIDE = 32;      // output tile side of the forward/proposal kernel

struct TileDesc {
    Frame f;
    State S;
    MomentBufs M;
    Prior pr;
    int burn_in;
    int B;                         // block side of the phase scan
    int series;                    // 0: block-phase pass, 1: block-series pass (B in [s - 1, s]),
                                   // 2: nine-phase block-series pass (B in [(s - 1)/2, s])
    int count[NLEV];               // items per level (per chain)
};

struct Item {
    int tile, chain, level, index;
};

// BK_WAVE<n>: nine-phase block-series items with up to n footprint entries per lane
enum BatchKind { BK_FORWARD = 0, BK_SERIES = 1, BK_PHASE = 2, BK_MOMENTS = 3, BK_FINALIZE = 4, BK_WAVE4 = 5,
                 BK_WAVE8 = 6, BK_WAVE16 = 7, BK_PHASE_EM = 8, BK_MOMENTS_EM = 9, BK_KINDS = 10 };
hipError_t launch_batch_level(int kind, const TileDesc* tiles, const Item* items, int n_items,
                              const double* inv_tab, size_t lds, hipStream_t st);
hipError_t launch_batch_advance(int64_t* const* tps, int n, hipStream_t st);
size_t forward_lds(int s);

}  // namespace bdc
