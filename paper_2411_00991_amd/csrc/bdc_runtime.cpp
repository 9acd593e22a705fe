// bdc_runtime.cpp -- host runtime behind the C ABI of include/bdc.h.
//
// Owns the device buffers of one frame, validates every input, orders its
// work after the caller's stream (event in, event out) on a private stream,
// and replays one captured sweep as a HIP graph.  No exception crosses the
// ABI: every entry point catches and maps failures to a bdc_status.
#include "../../include/bdc.h"
#include "../../include/bdc_unet.h"
#include "bdc_kernels.h"
#include "unet_net.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace bdc;

namespace {

thread_local std::string g_err = "no error";

struct Fail {
    bdc_status st;
    std::string msg;
};

[[noreturn]] void fail(bdc_status st, const std::string& msg) { throw Fail{st, msg}; }

void hipck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(BDC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(BDC_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return static_cast<T*>(p);
}

}  // namespace

struct bdc_ctx {
    bdc_config cfg{};
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string err = "no error";

    bool has_psf = false, has_cam = false, ready = false;
    int s = 0, r = 0, sched = 0, B = 0;   // s, r: footprint side and radius on the pixel lattice
    int64_t N = 0;                        // object cells (k^2 * height * width)
    int sub = 1;                          // object cells per pixel side k
    int64_t Np = 0;                       // camera pixels (height * width)
    int C = 0;
    int cam_per_pixel = 0;
    int max_batches = 0;

    float* d_psf = nullptr;
    std::vector<double> h_psf;         // normalised PSF (host copy, for the prior's OTF)
    uint16_t* d_psf_order = nullptr;   // footprint offsets by descending PSF weight
    // Dirichlet-OTF prior per chunk (prior_kind DIRICHLET)
    float* d_dir_am1 = nullptr;        // [4][B*B] alpha - 1 per chunk shape
    double* d_dir_const = nullptr;     // [4]
    double2* d_dir_F = nullptr;        // [C][N] chunk spectra
    double* d_dir_part = nullptr;      // [chunks][C] chunk log priors
    int dir_B = 0;
    // thinned sample export: [cap][C][N]
    float* d_samples = nullptr;
    int exp_thin = 0, exp_cap = 0;
    float* d_probs = nullptr;          // quantile levels of the last bdc_quantiles call
    int n_probs_alloc = 0;
    float* d_qout = nullptr;           // quantile output staging (host outputs)
    int64_t qout_alloc = 0;
    float4* d_pc = nullptr;
    float *d_w = nullptr, *d_gain = nullptr, *d_off = nullptr, *d_sig = nullptr;
    double* d_inv = nullptr;
    float *d_rho = nullptr, *d_ls = nullptr, *d_mu = nullptr;
    float *d_prho = nullptr, *d_phast = nullptr, *d_plogu = nullptr;
    int64_t* d_t = nullptr;
    unsigned long long* d_acc = nullptr;
    float *d_mean = nullptr, *d_m2 = nullptr, *d_batch = nullptr;
    double *d_lp = nullptr, *d_trace = nullptr;
    int* d_bad = nullptr;
    float* d_tmp = nullptr;          // N floats
    float* d_tmp2 = nullptr;         // N floats
    double* d_tmpd = nullptr;        // N doubles
    unsigned* d_hist = nullptr;
    float* d_dbg_delta = nullptr;    // C*N, lazily
    uint8_t* d_dbg_acc = nullptr;

    unsigned long long* d_ctr = nullptr;  // [0] phi terms, [1] footprint evaluations, [2] direct, [3] anchors, [4] anchor terms, [5] fused anchors

    // learned part: block-proposal maps, block-move counters
    float *d_pm = nullptr, *d_ps = nullptr;
    float* d_scale = nullptr;
    unsigned long long* d_bacc = nullptr;
    float* d_bdbg = nullptr;         // per-block debug deltas (C * N bound)
    uint8_t* d_bdbg_acc = nullptr;
    bool has_maps = false;
    float block_beta = 1.0f;
    float block_walk = 0.0f;         // > 0: block moves are the walk along what the blur removes
    int64_t block_pass = 0, block_proposed = 0;

    int64_t gen = 0;                 // bumped when the PSF or camera buffers change
    int64_t t = 0;                   // host shadow of the sweep index
    hipGraphExec_t graph = nullptr;
    bool use_graph = true;
    bool profiling = false;
    // measurement marks: event recorded after a kernel of class k (-1 = sweep start)
    std::vector<std::pair<hipEvent_t, int>> marks;

    Frame frame() const {
        Frame f;
        f.H = cfg.height * sub; f.W = cfg.width * sub; f.s = s; f.r = r; f.N = N; f.C = C;
        f.sub = sub; f.Hp = cfg.height; f.Wp = cfg.width; f.Np = Np;
        f.psf = d_psf; f.psf_order = d_psf_order; f.pc = d_pc; f.w = d_w; f.gain = d_gain; f.offset = d_off; f.sigma = d_sig;
        f.cam_per_pixel = cam_per_pixel;
        f.camera = cfg.camera;
        f.key = make_uint2((uint32_t)cfg.seed, (uint32_t)(cfg.seed >> 32));
        if (cfg.prior_kind == BDC_PRIOR_DIRICHLET && d_dir_am1) {
            f.dir_am1 = d_dir_am1;
            f.dir_const = d_dir_const;
            f.dir_F = d_dir_F;
            f.dir_B = dir_B;
        }
        return f;
    }
    State state() const {
        State S;
        S.rho = d_rho; S.log_step = d_ls; S.mu = d_mu;
        S.prop_rho = d_prho; S.prop_hast = d_phast; S.prop_logu = d_plogu;
        S.t = d_t; S.accepts = d_acc; S.counters = d_ctr;
        return S;
    }
    Prior prior() const { return Prior{cfg.prior_kind, cfg.prior_a, cfg.prior_b}; }
    MomentBufs moments() const {
        MomentBufs M;
        M.mean = d_mean; M.m2 = d_m2; M.batch = d_batch; M.rhat_block = cfg.rhat_block;
        M.max_batches = max_batches; M.lp_partial = d_lp; M.trace = d_trace; M.max_sweeps = cfg.max_sweeps;
        if (cfg.prior_kind == BDC_PRIOR_DIRICHLET && d_dir_part) {
            M.dir_part = d_dir_part;
            M.n_chunks = ((cfg.height + dir_B - 1) / dir_B) * ((cfg.width + dir_B - 1) / dir_B);
        }
        return M;
    }

    void enter() {
        hipck(hipEventRecord(ev_in, user), "hipEventRecord");
        hipck(hipStreamWaitEvent(work, ev_in, 0), "hipStreamWaitEvent");
    }
    void leave() {
        hipck(hipEventRecord(ev_out, work), "hipEventRecord");
        hipck(hipStreamWaitEvent(user, ev_out, 0), "hipStreamWaitEvent");
    }
    void sync() { hipck(hipStreamSynchronize(work), "hipStreamSynchronize"); }

    void drop_graph() {
        if (graph) { (void)hipGraphExecDestroy(graph); graph = nullptr; }
    }
    void clear_marks() {
        for (auto& m : marks) (void)hipEventDestroy(m.first);
        marks.clear();
    }
    void mark(int cls) {
        if (!profiling) return;
        hipEvent_t e;
        hipck(hipEventCreate(&e), "hipEventCreate");
        marks.emplace_back(e, cls);
        hipck(hipEventRecord(e, work), "hipEventRecord");
    }
    void free_all() {
        clear_marks();
        drop_graph();
        void* ptrs[] = {d_psf, d_psf_order, d_pc, d_w, d_gain, d_off, d_sig, d_inv, d_rho, d_ls, d_mu, d_prho, d_phast,
                        d_plogu, d_t, d_acc, d_mean, d_m2, d_batch, d_lp, d_trace, d_bad, d_tmp, d_tmp2,
                        d_tmpd, d_hist, d_dbg_delta, d_dbg_acc, d_ctr, d_pm, d_ps, d_scale, d_bacc,
                        d_bdbg, d_bdbg_acc, d_dir_am1, d_dir_const, d_dir_F, d_dir_part, d_samples, d_probs,
                        d_qout};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (work) (void)hipStreamDestroy(work);
    }
};

namespace {

// R-hat histogram: [0.9, 1.5) in 1e-5 bins, [1.5, 11.5) in 1e-3 bins, overflow
constexpr int HIST_FINE = 60000, HIST_COARSE = 10000, HIST_BINS = HIST_FINE + HIST_COARSE + 1;
constexpr float HIST_LO = 0.9f, HIST_W = 1e-5f, HIST_WC = 1e-3f;

// Copies n elements of T from a caller pointer into a host vector.
template <class T>
std::vector<T> fetch(bdc_ctx* c, const T* src, size_t n, int on_device) {
    std::vector<T> v(n);
    if (n == 0) return v;
    if (on_device) {
        hipck(hipMemcpyAsync(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, c->work), "hipMemcpyAsync D2H");
        c->sync();
    } else {
        std::memcpy(v.data(), src, n * sizeof(T));
    }
    return v;
}

void download(bdc_ctx* c, void* dst, const void* src, size_t bytes, int on_device) {
    hipck(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->work),
          "hipMemcpyAsync download");
}

void set_t(bdc_ctx* c, int64_t t) {
    c->t = t;
    static_assert(sizeof(int64_t) == 8, "");
    hipck(hipMemcpyAsync(c->d_t, &c->t, sizeof(int64_t), hipMemcpyHostToDevice, c->work), "set sweep index");
    c->sync();
}

void check_finite(const std::vector<float>& v, const char* what) {
    for (float x : v)
        if (!std::isfinite(x)) fail(BDC_ENOTFINITE, std::string(what) + " holds NaN or Inf");
}

void need(bdc_ctx* c, bool cond, bdc_status st, const char* msg) {
    (void)c;
    if (!cond) fail(st, msg);
}

// Entry points that work on the pixel lattice only (object_sub <= 1).
void pixel_lattice_only(bdc_ctx* c, const char* what) {
    if (c->sub > 1) fail(BDC_EINVAL, std::string(what) + " needs object lattice = pixel lattice (object_sub <= 1)");
}

void choose_schedule(bdc_ctx* c) {
    const int s = c->s;
    int sched = c->cfg.schedule;
    int B = c->cfg.block_size;
    if (c->sub > 1) {
        // a finer object lattice: the pixel-chromatic or the block-phase scan
        // over cell phases (B in pixels; s is the pixel-footprint side)
        if (sched != BDC_SCHED_AUTO && sched != BDC_SCHED_CHROMATIC && sched != BDC_SCHED_BLOCK)
            fail(BDC_EINVAL, "a finer object lattice runs the pixel-chromatic or the block-phase scan");
        const int Bd = B == 0 ? std::max(s, std::min(4 * s, 8)) : B;
        const bool fits = Bd >= std::max(1, s - 1) && Bd <= 4 * s &&
                          block_phase_sub_lds(Bd, s, c->sub) <= 64 * 1024;
        if (sched == BDC_SCHED_AUTO)
            sched = std::min(c->cfg.height, c->cfg.width) >= 2 * s && fits ? BDC_SCHED_BLOCK : BDC_SCHED_CHROMATIC;
        if (sched == BDC_SCHED_BLOCK && !fits)
            fail(BDC_EINVAL, "block_size must lie in [footprint side - 1, 4 * footprint side] (pixels) and the "
                             "footprint tables and region fit 64 KiB of LDS");
        c->sched = sched;
        c->B = sched == BDC_SCHED_BLOCK ? Bd : 0;
        return;
    }
    if (c->cfg.prior_kind == BDC_PRIOR_DIRICHLET) {
        // the prior couples the pixels of a chunk (a block): one pixel per block
        // and colour, B in [s - 1, s]
        if (sched != BDC_SCHED_AUTO && sched != BDC_SCHED_BLOCK)
            fail(BDC_EINVAL, "the Dirichlet-OTF prior runs with the block-phase scan");
        if (B == 0) B = s;
        if (s > 31 || B > s || B < std::max(1, s - 1))
            fail(BDC_EINVAL, "the Dirichlet-OTF prior needs a PSF side <= 31 and block_size in [psf side - 1, "
                             "psf side]");
        c->sched = BDC_SCHED_BLOCK;
        c->B = B;
        return;
    }
    if (c->cfg.camera == BDC_CAMERA_EMCCD) {
        // the truncation-bounded local series is derived for the sCMOS reading;
        // an EMCCD pixel's likelihood change is the closed form in every pass
        if (sched == BDC_SCHED_BLOCK_SERIES || sched == BDC_SCHED_BLOCK9_SERIES)
            fail(BDC_EINVAL, "the block-series scans take the sCMOS reading only");
        if (sched == BDC_SCHED_AUTO)
            sched = std::min(c->cfg.height, c->cfg.width) < 2 * s ? BDC_SCHED_CHROMATIC : BDC_SCHED_BLOCK;
    }
    if (sched == BDC_SCHED_AUTO) {
        // measured on MI355X (1024^2 and 2048^2 frames, 4 chains): the
        // one-wavefront nine-phase pass is the faster series pass up to PSF
        // side 21 (B = s up to side 11, about half the side above), the
        // four-wave pass beyond
        const int B9 = s <= 11 ? s : std::max(1, s / 2);
        if (std::min(c->cfg.height, c->cfg.width) < 2 * s) sched = BDC_SCHED_CHROMATIC;
        else if (B == 0 && s <= 21 && wave_series_fits(B9, s)) {
            sched = BDC_SCHED_BLOCK9_SERIES;
            B = B9;
        } else if (B == 0 && block_series_fits(std::max(1, s - 1), s)) sched = BDC_SCHED_BLOCK_SERIES;
        else if (B != 0 && block_series_fits(B, s)) sched = BDC_SCHED_BLOCK_SERIES;
        else sched = BDC_SCHED_BLOCK;
    }
    if (sched == BDC_SCHED_BLOCK) {
        if (B == 0) B = std::max(s, std::min(4 * s, 8));
        if (B < s - 1 || B > 4 * s || B < 1) fail(BDC_EINVAL, "block_size must lie in [psf side - 1, 4 * psf side]");
        if (block_phase_lds(B, s) > 64 * 1024) fail(BDC_EINVAL, "block_size too large for 64 KiB of LDS");
    } else if (sched == BDC_SCHED_BLOCK_SERIES) {
        // B = s - 1 measured 1 % faster than B = s at 2048^2 with the Airy 31 x 31 PSF
        if (B == 0) B = std::max(1, s - 1);
        if (!block_series_fits(B, s))
            fail(BDC_EINVAL, "the block-series scan needs block_size in [psf side - 1, psf side] and a PSF of "
                             "at most 32 x 32");
    } else if (sched == BDC_SCHED_BLOCK9_SERIES) {
        if (B == 0) B = std::max(1, s / 2);
        if (!wave_series_fits(B, s))
            fail(BDC_EINVAL, "the nine-phase block-series scan needs block_size in [(psf side - 1) / 2, psf side] "
                             "and a PSF of at most 32 x 32");
    } else if (sched != BDC_SCHED_CHROMATIC) {
        fail(BDC_EINVAL, "unknown schedule");
    }
    c->sched = sched;
    c->B = B;
}

// Dirichlet-OTF prior tables (Methods, Prior, Eq. 8) for the chunk shapes of
// the frame: alpha = |OTF| / sum |OTF| with the OTF the DFT of the PSF wrapped
// onto the chunk grid (centre at index 0), floored at 1e-6 / K and
// renormalised; stored as alpha - 1 with the constant lgamma(sum alpha) -
// sum_k lgamma(alpha_k) of each shape.  Chunk spectra and log priors buffers.
void build_dirichlet(bdc_ctx* c) {
    if (c->cfg.prior_kind != BDC_PRIOR_DIRICHLET) return;
    const int B = c->B, s = c->s, r = s / 2;
    const int eh = c->cfg.height % B ? c->cfg.height % B : B, ew = c->cfg.width % B ? c->cfg.width % B : B;
    std::vector<float> am(4 * (size_t)B * B, 0.0f);
    double cst[4];
    for (int shape = 0; shape < 4; ++shape) {
        const int th = (shape & 2) ? eh : B, tw = (shape & 1) ? ew : B, K = th * tw;
        std::vector<double> wr(K, 0.0), a(K);
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx)
                wr[((dy % th + th) % th) * tw + ((dx % tw + tw) % tw)] += c->h_psf[(dy + r) * s + (dx + r)];
        double tot = 0.0;
        for (int ky = 0; ky < th; ++ky)
            for (int kx = 0; kx < tw; ++kx) {
                double re = 0.0, im = 0.0;
                for (int y = 0; y < th; ++y)
                    for (int x = 0; x < tw; ++x) {
                        const double ang = 2.0 * M_PI * ((double)((ky * y) % th) / th + (double)((kx * x) % tw) / tw);
                        re += wr[y * tw + x] * std::cos(ang);
                        im -= wr[y * tw + x] * std::sin(ang);
                    }
                a[ky * tw + kx] = std::sqrt(re * re + im * im);
                tot += a[ky * tw + kx];
            }
        double tot2 = 0.0;
        for (int k = 0; k < K; ++k) {
            a[k] = std::max(a[k] / tot, 1e-6 / K);
            tot2 += a[k];
        }
        double lg = 0.0, asum = 0.0;
        for (int k = 0; k < K; ++k) {
            a[k] /= tot2;
            asum += a[k];
            lg -= std::lgamma(a[k]);
            am[(size_t)shape * B * B + k] = (float)(a[k] - 1.0);
        }
        cst[shape] = lg + std::lgamma(asum);
    }
    const size_t CN = (size_t)c->C * c->N;
    const int nch = ((c->cfg.height + B - 1) / B) * ((c->cfg.width + B - 1) / B);
    for (void** p : {(void**)&c->d_dir_am1, (void**)&c->d_dir_const, (void**)&c->d_dir_F, (void**)&c->d_dir_part})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    c->d_dir_am1 = dalloc<float>(am.size());
    c->d_dir_const = dalloc<double>(4);
    c->d_dir_F = dalloc<double2>(CN);
    c->d_dir_part = dalloc<double>((size_t)nch * c->C);
    hipck(hipMemcpy(c->d_dir_am1, am.data(), am.size() * sizeof(float), hipMemcpyHostToDevice), "upload alpha");
    hipck(hipMemcpy(c->d_dir_const, cst, sizeof(cst), hipMemcpyHostToDevice), "upload alpha constants");
    c->dir_B = B;
}

void run_sweep_body(bdc_ctx* c, hipStream_t st) {
    const Frame f = c->frame();
    const State S = c->state();
    c->mark(-1);
    hipck(launch_forward_propose(f, S, c->prior(), 1, st), "forward_propose");
    hipck(launch_chunk_spectra(f, S, st), "chunk_spectra");
    c->mark(0);
    if (c->sched == BDC_SCHED_CHROMATIC) {
        for (int k = 0; k < c->sub * c->sub * c->s * c->s; ++k) {
            hipck(launch_colour_pass(f, S, c->cfg.burn_in, c->d_inv, k, nullptr, nullptr, st), "colour_pass");
            c->mark(1);
        }
    } else if (c->sched == BDC_SCHED_BLOCK_SERIES) {
        for (int ph = 0; ph < 4; ++ph) {
            hipck(launch_block_series(f, S, c->cfg.burn_in, c->d_inv, c->B, ph, 0, c->s * c->s, nullptr, nullptr, st),
                  "block_series");
            c->mark(1);
        }
    } else if (c->sched == BDC_SCHED_BLOCK9_SERIES) {
        for (int ph = 0; ph < 9; ++ph) {
            hipck(launch_wave_series(f, S, c->cfg.burn_in, c->B, ph, 0, c->s * c->s, nullptr, nullptr, st),
                  "wave_series");
            c->mark(1);
        }
    } else {
        for (int ph = 0; ph < 4; ++ph) {
            hipck(launch_block_phase(f, S, c->cfg.burn_in, c->d_inv, c->B, ph, 0, c->sub * c->sub * c->s * c->s,
                                     nullptr, nullptr, st),
                  "block_phase");
            c->mark(1);
        }
    }
    if (c->d_samples)
        hipck(launch_export(f, c->d_rho, c->d_t, c->cfg.burn_in, c->exp_thin, c->exp_cap, c->d_samples, st),
              "export");
    hipck(launch_moments(f, S, c->prior(), c->moments(), c->cfg.burn_in, 1, st), "moments");
    c->mark(2);
}

void build_graph(bdc_ctx* c) {
    c->drop_graph();
    hipGraph_t g = nullptr;
    hipck(hipStreamBeginCapture(c->work, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        run_sweep_body(c, c->work);
    } catch (...) {
        (void)hipStreamEndCapture(c->work, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipck(hipStreamEndCapture(c->work, &g), "hipStreamEndCapture");
    hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hipck(e, "hipGraphInstantiate");
}

template <class F>
bdc_status guarded(bdc_ctx* c, F&& fn) {
    try {
        fn();
        if (c) c->err = "no error";
        return BDC_OK;
    } catch (const Fail& f) {
        if (c) c->err = f.msg; else g_err = f.msg;
        return f.st;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed"; else g_err = "host allocation failed";
        return BDC_ENOMEM;
    } catch (...) {
        if (c) c->err = "unexpected internal error"; else g_err = "unexpected internal error";
        return BDC_EDEVICE;
    }
}

// Windows of the diagnostics (host arithmetic): a batch counts once all its
// rhat_block sweeps have run and lie inside the max_sweeps store, so every
// window stays inside the batch store and the log-posterior trace.
static bdc_status diag_window(const bdc_config& k, int64_t t, int* b_lo, int* half, int* b0, int* nb) {
    const int rb = k.rhat_block > 0 ? k.rhat_block : 25;
    const int ms = k.max_sweeps > 0 ? k.max_sweeps : 4096;
    if (t < 0 || t > ms) return BDC_ESTATE;
    const int done = (int)(t / rb);                 // complete batches, all inside the store
    const int h = done / 4;
    if (half) *half = h;
    if (b_lo) *b_lo = done - 2 * h;
    const int first = (std::max(k.burn_in, 0) + rb - 1) / rb;
    if (b0) *b0 = first;
    if (nb) *nb = std::max(done - first, 0);
    return BDC_OK;
}

// Samples stored by the export after t sweeps: post-burn-in sweeps whose index
// is a multiple of thin past burn_in, at most cap.
static int64_t stored_samples(int64_t t, int burn_in, int thin, int cap) {
    if (thin < 1 || t <= burn_in) return 0;
    return std::min<int64_t>((t - burn_in + thin - 1) / thin, cap);
}

struct StateHeader {
    uint64_t magic;
    int32_t H, W, C, s;
    int64_t t;
    int32_t nb, rhat_block;
    int32_t sub, reserved;         // object cells per pixel side (rho is k^2 H W per chain)
    int64_t n_trace;
};
constexpr uint64_t STATE_MAGIC = 0x3230303143444231ull;  // "1BDC1002"

}  // namespace

extern "C" {

bdc_status bdc_diag_window(const bdc_config* cfg, int64_t t, int32_t* b_lo, int32_t* half, int32_t* b0,
                           int32_t* nb) {
    if (!cfg) return BDC_EINVAL;
    if (cfg->rhat_block < 0 || cfg->max_sweeps < 0) return BDC_EINVAL;
    int a = 0, h = 0, f = 0, n = 0;
    const bdc_status st = diag_window(*cfg, t, &a, &h, &f, &n);
    if (st != BDC_OK) return st;
    if (b_lo) *b_lo = a;
    if (half) *half = h;
    if (b0) *b0 = f;
    if (nb) *nb = n;
    return BDC_OK;
}

void bdc_config_default(bdc_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_chains = 1;
    cfg->prior_kind = BDC_PRIOR_FLAT;
    cfg->prior_a = 1.0f;
    cfg->prior_b = 0.0f;
    cfg->log_step0 = -1.5f;
    cfg->schedule = BDC_SCHED_AUTO;
    cfg->rhat_block = 25;
    cfg->max_sweeps = 4096;
}

bdc_status bdc_create(const bdc_config* cfg, void* hip_stream, bdc_ctx** out) {
    if (!out) { g_err = "out is NULL"; return BDC_EINVAL; }
    *out = nullptr;
    bdc_ctx* c = nullptr;
    bdc_status st = guarded(nullptr, [&] {
        if (!cfg) fail(BDC_EINVAL, "cfg is NULL");
        bdc_config k = *cfg;
        if (k.rhat_block == 0) k.rhat_block = 25;
        if (k.max_sweeps == 0) k.max_sweeps = 4096;
        if (k.height < 1 || k.width < 1 || k.height > 32768 || k.width > 32768)
            fail(BDC_EINVAL, "height and width must lie in [1, 32768]");
        if ((int64_t)k.height * k.width > (1ll << 27)) fail(BDC_EINVAL, "frame larger than 2^27 pixels");
        if (k.n_chains < 1 || k.n_chains > 64) fail(BDC_EINVAL, "n_chains must lie in [1, 64]");
        if (k.prior_kind != BDC_PRIOR_FLAT && k.prior_kind != BDC_PRIOR_GAMMA && k.prior_kind != BDC_PRIOR_DIRICHLET)
            fail(BDC_EINVAL, "unknown prior_kind");
        if (k.prior_kind == BDC_PRIOR_GAMMA && (!(k.prior_a > 0.0f) || !(k.prior_b >= 0.0f) ||
                                                !std::isfinite(k.prior_a) || !std::isfinite(k.prior_b)))
            fail(BDC_EINVAL, "Gamma prior needs shape > 0 and rate >= 0");
        if (k.burn_in < 0) fail(BDC_EINVAL, "burn_in must be >= 0");
        if (!std::isfinite(k.log_step0)) fail(BDC_ENOTFINITE, "log_step0 is not finite");
        if (k.schedule < 0 || k.schedule > 4) fail(BDC_EINVAL, "unknown schedule");
        if (k.camera != BDC_CAMERA_SCMOS && k.camera != BDC_CAMERA_EMCCD) fail(BDC_EINVAL, "unknown camera");
        if (k.block_size < 0) fail(BDC_EINVAL, "block_size must be >= 0");
        if (k.rhat_block < 1 || k.max_sweeps < 1) fail(BDC_EINVAL, "rhat_block and max_sweeps must be >= 1");
        if (k.object_sub < 0 || k.object_sub > 4) fail(BDC_EINVAL, "object_sub must lie in [0, 4]");
        const int sub = std::max(1, (int)k.object_sub);
        if ((int64_t)k.height * k.width * sub * sub > (1ll << 27)) fail(BDC_EINVAL, "object lattice larger than 2^27 cells");
        if (sub > 1 && k.prior_kind == BDC_PRIOR_DIRICHLET)
            fail(BDC_EINVAL, "the Dirichlet-OTF prior takes object lattice = pixel lattice");
        if (sub > 1 && k.schedule != BDC_SCHED_AUTO && k.schedule != BDC_SCHED_CHROMATIC &&
            k.schedule != BDC_SCHED_BLOCK)
            fail(BDC_EINVAL, "a finer object lattice runs the pixel-chromatic or the block-phase scan");
        c = new bdc_ctx();
        c->cfg = k;
        c->user = (hipStream_t)hip_stream;
        c->sub = sub;
        c->Np = (int64_t)k.height * k.width;
        c->N = c->Np * sub * sub;
        c->C = k.n_chains;
        c->max_batches = (k.max_sweeps + k.rhat_block - 1) / k.rhat_block;
        const char* ng = std::getenv("BDC_NO_GRAPH");
        c->use_graph = !(ng && ng[0] == '1');
        hipck(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking), "hipStreamCreate");
        hipck(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming), "hipEventCreate");
        hipck(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming), "hipEventCreate");
        const size_t CN = (size_t)c->C * c->N;
        c->d_pc = dalloc<float4>((size_t)c->Np);
        c->d_w = dalloc<float>(c->Np);
        c->d_rho = dalloc<float>(CN);
        c->d_ls = dalloc<float>(CN);
        c->d_mu = dalloc<float>((size_t)c->C * c->Np);
        c->d_prho = dalloc<float>(CN);
        c->d_phast = dalloc<float>(CN);
        c->d_plogu = dalloc<float>(CN);
        c->d_t = dalloc<int64_t>(1);
        c->d_acc = dalloc<unsigned long long>(c->C);
        c->d_mean = dalloc<float>(CN);
        c->d_m2 = dalloc<float>(CN);
        c->d_batch = dalloc<float>((size_t)c->max_batches * 3 * CN);
        c->d_lp = dalloc<double>((size_t)((c->N + WG - 1) / WG) * c->C);
        c->d_trace = dalloc<double>((size_t)k.max_sweeps * c->C);
        c->d_bad = dalloc<int>(4);
        c->d_tmp = dalloc<float>(c->N);
        c->d_tmp2 = dalloc<float>(c->N);
        c->d_tmpd = dalloc<double>(c->N);
        c->d_hist = dalloc<unsigned>(HIST_BINS);
        c->d_ctr = dalloc<unsigned long long>(NCOUNTERS);
        hipck(hipMemset(c->d_ctr, 0, NCOUNTERS * sizeof(unsigned long long)), "hipMemset");
        std::vector<double> inv(INV_TABLE);
        inv[0] = 0.0;
        for (int i = 1; i < INV_TABLE; ++i) inv[i] = 1.0 / (double)i;
        c->d_inv = dalloc<double>(INV_TABLE);
        hipck(hipMemcpy(c->d_inv, inv.data(), INV_TABLE * sizeof(double), hipMemcpyHostToDevice), "upload table");
    });
    if (st != BDC_OK) {
        if (c) { c->free_all(); delete c; }
        return st;
    }
    *out = c;
    return BDC_OK;
}

bdc_status bdc_set_psf(bdc_ctx* c, const float* psf, int32_t ph, int32_t pw, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, psf != nullptr, BDC_EINVAL, "psf is NULL");
        need(c, ph == pw && ph >= 1 && ph % 2 == 1 && ph <= 63, BDC_EINVAL, "PSF must be square with an odd side <= 63");
        const int F = ph * pw;
        std::vector<float> h = fetch(c, psf, F, on_device);
        double tot = 0.0;
        for (float v : h) {
            if (!std::isfinite(v)) fail(BDC_ENOTFINITE, "PSF holds NaN or Inf");
            if (v < 0.0f) fail(BDC_EINVAL, "PSF has a negative entry");
            tot += v;
        }
        need(c, tot > 0.0, BDC_EINVAL, "PSF sums to zero");
        std::vector<float> nrm(F);
        for (int i = 0; i < F; ++i) nrm[i] = (float)((double)h[i] / tot);
        c->sync();
        if (c->d_psf) { (void)hipFree(c->d_psf); c->d_psf = nullptr; }
        if (c->sub > 1) {
            // finer object lattice (Eqs. 1-2): the PSF is sampled on the object
            // lattice; a cell of phase (a, b) in pixel p sends to pixel p + d the
            // PSF summed over the offsets from the cell to the k x k cells of
            // p + d, T[a k + b][d] = sum_{i,j < k} P(d_y k + i - a, d_x k + j - b),
            // nonzero for |d| <= rp = floor((r + k - 1) / k)
            const int k = c->sub, ro = ph / 2, rp = (ro + k - 1) / k, sp = 2 * rp + 1;
            std::vector<float> tab((size_t)k * k * sp * sp);
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b)
                    for (int dy = -rp; dy <= rp; ++dy)
                        for (int dx = -rp; dx <= rp; ++dx) {
                            double acc = 0.0;
                            for (int i = 0; i < k; ++i)
                                for (int j = 0; j < k; ++j) {
                                    const int oy = dy * k + i - a, ox = dx * k + j - b;
                                    if (oy < -ro || oy > ro || ox < -ro || ox > ro) continue;
                                    acc += (double)h[(oy + ro) * ph + (ox + ro)] / tot;
                                }
                            tab[((size_t)(a * k + b) * sp + (dy + rp)) * sp + (dx + rp)] = (float)acc;
                        }
            c->d_psf = dalloc<float>(tab.size());
            hipck(hipMemcpy(c->d_psf, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice), "upload PSF");
            if (c->d_psf_order) { (void)hipFree(c->d_psf_order); c->d_psf_order = nullptr; }
            c->s = sp;
            c->r = rp;
            c->h_psf.assign(F, 0.0);
            for (int i = 0; i < F; ++i) c->h_psf[i] = (double)h[i] / tot;
            choose_schedule(c);
            c->has_psf = true;
            c->gen++;
            c->ready = false;
            c->drop_graph();
            return;
        }
        c->d_psf = dalloc<float>(F);
        hipck(hipMemcpy(c->d_psf, nrm.data(), F * sizeof(float), hipMemcpyHostToDevice), "upload PSF");
        // footprint offsets for the block-series pass in descending PSF weight
        // (ties by index): each thread's first entry covers the PSF core, where
        // moves are large, and the heaviest 64 fall on the first wave, so direct
        // evaluations concentrate on one wave
        std::vector<uint16_t> order(F);
        for (int i = 0; i < F; ++i) order[i] = (uint16_t)i;
        std::stable_sort(order.begin(), order.end(), [&](uint16_t a, uint16_t b) { return nrm[a] > nrm[b]; });
        if (c->d_psf_order) { (void)hipFree(c->d_psf_order); c->d_psf_order = nullptr; }
        c->d_psf_order = dalloc<uint16_t>(F);
        hipck(hipMemcpy(c->d_psf_order, order.data(), F * sizeof(uint16_t), hipMemcpyHostToDevice), "upload order");
        c->s = ph;
        c->r = ph / 2;
        c->h_psf.assign(F, 0.0);
        for (int i = 0; i < F; ++i) c->h_psf[i] = (double)h[i] / tot;
        choose_schedule(c);
        build_dirichlet(c);
        c->has_psf = true;
        c->gen++;
        c->ready = false;
        c->drop_graph();
    });
}

bdc_status bdc_set_camera_maps(bdc_ctx* c, const float* gain, const float* offset, const float* sigma,
                               int32_t per_pixel, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, gain && offset && sigma, BDC_EINVAL, "camera pointer is NULL");
        const size_t n = per_pixel ? (size_t)c->Np : 1;
        std::vector<float> g = fetch(c, gain, n, on_device);
        std::vector<float> o = fetch(c, offset, n, on_device);
        std::vector<float> sg = fetch(c, sigma, n, on_device);
        check_finite(g, "gain");
        check_finite(o, "offset");
        check_finite(sg, "read_sigma");
        for (size_t i = 0; i < n; ++i)
            if (!(g[i] > 0.0f) || !(sg[i] > 0.0f)) fail(BDC_EINVAL, "gain and read_sigma must be > 0");
        c->sync();
        for (float** p : {&c->d_gain, &c->d_off, &c->d_sig})
            if (*p) { (void)hipFree(*p); *p = nullptr; }
        c->d_gain = dalloc<float>(n);
        c->d_off = dalloc<float>(n);
        c->d_sig = dalloc<float>(n);
        hipck(hipMemcpy(c->d_gain, g.data(), n * sizeof(float), hipMemcpyHostToDevice), "upload gain");
        hipck(hipMemcpy(c->d_off, o.data(), n * sizeof(float), hipMemcpyHostToDevice), "upload offset");
        hipck(hipMemcpy(c->d_sig, sg.data(), n * sizeof(float), hipMemcpyHostToDevice), "upload sigma");
        c->cam_per_pixel = per_pixel ? 1 : 0;
        c->has_cam = true;
        c->gen++;
        c->ready = false;
        c->drop_graph();
    });
}

bdc_status bdc_init(bdc_ctx* c, const float* image, const float* rho0, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->has_psf && c->has_cam, BDC_ESTATE, "set_psf and set_camera_maps must precede init");
        need(c, image != nullptr, BDC_EINVAL, "image is NULL");
        c->enter();
        std::vector<float> w = fetch(c, image, (size_t)c->Np, on_device);
        check_finite(w, "image");
        hipck(hipMemcpyAsync(c->d_w, w.data(), c->Np * sizeof(float), hipMemcpyHostToDevice, c->work), "upload image");
        hipck(hipMemsetAsync(c->d_bad, 0, 4 * sizeof(int), c->work), "hipMemsetAsync");
        const Frame f = c->frame();
        hipck(launch_pixel_consts(f, c->d_pc, c->d_bad, c->work), "pixel_consts");
        const size_t CN = (size_t)c->C * c->N;
        const float* r0 = nullptr;
        if (rho0) {
            if (on_device) {
                r0 = rho0;
            } else {
                hipck(hipMemcpyAsync(c->d_prho, rho0, CN * sizeof(float), hipMemcpyHostToDevice, c->work), "upload rho0");
                r0 = c->d_prho;
            }
        }
        hipck(launch_init_state(f, c->state(), r0, c->cfg.log_step0, c->d_bad + 2, c->work), "init_state");
        hipck(launch_fill_f32(c->d_mean, CN, 0.0f, c->work), "fill");
        hipck(launch_fill_f32(c->d_m2, CN, 0.0f, c->work), "fill");
        hipck(hipMemsetAsync(c->d_acc, 0, c->C * sizeof(unsigned long long), c->work), "hipMemsetAsync");
        int bad[4] = {0, 0, 0, 0};
        hipck(hipMemcpyAsync(bad, c->d_bad, sizeof(bad), hipMemcpyDeviceToHost, c->work), "read flags");
        c->sync();
        if (bad[0] > 0) fail(BDC_ENOTFINITE, "non-finite value in the frame or camera");
        if (bad[1] > 0) fail(BDC_EINVAL, "non-positive gain or read noise");
        if (bad[2] > 0) fail(BDC_EINVAL, "rho0 must be finite and > 0");
        set_t(c, 0);
        c->ready = true;
        c->leave();
    });
}

bdc_status bdc_sweep(bdc_ctx* c, int32_t n) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede sweep");
        need(c, n >= 0, BDC_EINVAL, "n must be >= 0");
        if (n == 0) return;
        c->enter();
        if (c->use_graph && !c->profiling) {
            if (!c->graph) build_graph(c);
            for (int i = 0; i < n; ++i) hipck(hipGraphLaunch(c->graph, c->work), "hipGraphLaunch");
        } else {
            for (int i = 0; i < n; ++i) run_sweep_body(c, c->work);
        }
        c->t += n;
        c->leave();
    });
}

bdc_status bdc_posterior_moments(bdc_ctx* c, int32_t chain, float* mean, float* var, int64_t* n_samples,
                                 int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede posterior_moments");
        need(c, chain >= -1 && chain < c->C, BDC_EINVAL, "chain out of range");
        const int64_t ns = std::max<int64_t>(0, c->t - c->cfg.burn_in);
        if (n_samples) *n_samples = ns;
        need(c, ns >= 2, BDC_ESTATE, "fewer than 2 post-burn-in sweeps");
        c->enter();
        hipck(launch_pooled_moments(c->frame(), c->moments(), ns, chain, mean ? c->d_tmp : nullptr,
                                    var ? c->d_tmp2 : nullptr, c->work), "pooled moments");
        if (mean) download(c, mean, c->d_tmp, c->N * sizeof(float), on_device);
        if (var) download(c, var, c->d_tmp2, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

static void rhat_window(bdc_ctx* c, int* b_lo, int* half) {
    if (diag_window(c->cfg, c->t, b_lo, half, nullptr, nullptr) != BDC_OK)
        fail(BDC_ESTATE, "more sweeps than max_sweeps: the diagnostics need every sweep in the batch store "
                         "(create the context with a larger max_sweeps)");
}

bdc_status bdc_rhat_map(bdc_ctx* c, float* rhat, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede rhat");
        need(c, c->C >= 2, BDC_ESTATE, "R-hat needs at least 2 chains");
        int b_lo, half;
        rhat_window(c, &b_lo, &half);
        need(c, half >= 1, BDC_ESTATE, "R-hat needs at least 4 completed batches");
        c->enter();
        hipck(launch_rhat_map(c->frame(), c->moments(), b_lo, half, c->d_tmp, c->work), "rhat map");
        if (rhat) download(c, rhat, c->d_tmp, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_window_mean(bdc_ctx* c, float* mean, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede window_mean");
        need(c, mean != nullptr, BDC_EINVAL, "mean is NULL");
        int b_lo, half;
        rhat_window(c, &b_lo, &half);
        need(c, half >= 1, BDC_ESTATE, "the window needs at least 4 completed batches");
        c->enter();
        hipck(launch_window_mean(c->frame(), c->moments(), b_lo, 2 * half, c->d_tmp, c->work), "window mean");
        download(c, mean, c->d_tmp, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_rhat(bdc_ctx* c, float* rhat_p99, float* rhat_logpost) {
    if (!c) return BDC_EINVAL;
    bdc_status st = bdc_rhat_map(c, nullptr, 0);
    if (st != BDC_OK) return st;
    return guarded(c, [&] {
        int b_lo, half;
        rhat_window(c, &b_lo, &half);
        c->enter();
        hipck(hipMemsetAsync(c->d_hist, 0, HIST_BINS * sizeof(unsigned), c->work), "hipMemsetAsync");
        hipck(launch_hist(c->d_tmp, c->N, HIST_LO, HIST_W, HIST_FINE, HIST_WC, HIST_COARSE, c->d_hist, c->work),
              "hist");
        std::vector<unsigned> h(HIST_BINS);
        hipck(hipMemcpyAsync(h.data(), c->d_hist, HIST_BINS * sizeof(unsigned), hipMemcpyDeviceToHost, c->work),
              "read hist");
        const int L = half * c->cfg.rhat_block;
        const int64_t t0 = (int64_t)b_lo * c->cfg.rhat_block;
        std::vector<double> tr((size_t)2 * L * c->C);
        hipck(hipMemcpyAsync(tr.data(), c->d_trace + t0 * c->C, tr.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->work), "read trace");
        c->sync();
        c->leave();
        if (rhat_p99) {
            const double target = 0.99 * (double)c->N;
            double cum = 0.0;
            int b = 0;
            for (; b < HIST_BINS; ++b) {
                cum += h[b];
                if (cum >= target) break;
            }
            if (b >= HIST_BINS - 1) *rhat_p99 = INFINITY;
            else if (b < HIST_FINE) *rhat_p99 = HIST_LO + (float)(b + 1) * HIST_W;
            else *rhat_p99 = HIST_LO + HIST_FINE * HIST_W + (float)(b - HIST_FINE + 1) * HIST_WC;
        }
        if (rhat_logpost) {
            // split R-hat of the trace over the same window (2C sequences of length L)
            const int m = 2 * c->C;
            double sm = 0.0, sm2 = 0.0, sv = 0.0;
            for (int ch = 0; ch < c->C; ++ch)
                for (int hh = 0; hh < 2; ++hh) {
                    double mean = 0.0;
                    for (int i = 0; i < L; ++i) mean += tr[(size_t)(hh * L + i) * c->C + ch];
                    mean /= L;
                    double v = 0.0;
                    for (int i = 0; i < L; ++i) {
                        const double d = tr[(size_t)(hh * L + i) * c->C + ch] - mean;
                        v += d * d;
                    }
                    v /= (L - 1);
                    sm += mean;
                    sm2 += mean * mean;
                    sv += v;
                }
            const double gm = sm / m;
            const double Bv = L * (sm2 - m * gm * gm) / (m - 1);
            const double Wv = sv / m;
            *rhat_logpost = (float)std::sqrt(((L - 1.0) / L * Wv + Bv / L) / Wv);
        }
    });
}

bdc_status bdc_mcse(bdc_ctx* c, float* mcse, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede mcse");
        need(c, mcse != nullptr, BDC_EINVAL, "mcse is NULL");
        int b0 = 0, nb = 0;
        if (diag_window(c->cfg, c->t, nullptr, nullptr, &b0, &nb) != BDC_OK)
            fail(BDC_ESTATE, "more sweeps than max_sweeps: the diagnostics need every sweep in the batch store "
                             "(create the context with a larger max_sweeps)");
        need(c, nb >= 2, BDC_ESTATE, "MCSE needs at least 2 post-burn-in batches");
        c->enter();
        hipck(launch_mcse(c->frame(), c->moments(), b0, nb, c->d_tmp, c->work), "mcse");
        download(c, mcse, c->d_tmp, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_get_rho(bdc_ctx* c, float* rho, float* log_step, int64_t* sweep, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede get_rho");
        c->enter();
        const size_t b = (size_t)c->C * c->N * sizeof(float);
        if (rho) download(c, rho, c->d_rho, b, on_device);
        if (log_step) download(c, log_step, c->d_ls, b, on_device);
        c->sync();
        if (sweep) *sweep = c->t;
        c->leave();
    });
}

bdc_status bdc_get_mu(bdc_ctx* c, float* mu, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede get_mu");
        need(c, mu != nullptr, BDC_EINVAL, "mu is NULL");
        c->enter();
        hipck(launch_forward_propose(c->frame(), c->state(), c->prior(), 0, c->work), "forward");
        download(c, mu, c->d_mu, (size_t)c->C * c->Np * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_loglik(bdc_ctx* c, int32_t chain, float* ell, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede loglik");
        need(c, chain >= 0 && chain < c->C, BDC_EINVAL, "chain out of range");
        need(c, ell != nullptr, BDC_EINVAL, "ell is NULL");
        c->enter();
        hipck(launch_forward_propose(c->frame(), c->state(), c->prior(), 0, c->work), "forward");
        hipck(launch_loglik(c->frame(), c->d_mu + (size_t)chain * c->Np, c->d_tmpd, c->work), "loglik");
        std::vector<double> h((size_t)c->Np);
        hipck(hipMemcpyAsync(h.data(), c->d_tmpd, c->Np * sizeof(double), hipMemcpyDeviceToHost, c->work), "read");
        c->sync();
        std::vector<float> hf((size_t)c->Np);
        for (int64_t i = 0; i < c->Np; ++i) hf[i] = (float)h[i];
        if (on_device) {
            hipck(hipMemcpyAsync(ell, hf.data(), c->Np * sizeof(float), hipMemcpyHostToDevice, c->work), "write");
            c->sync();
        } else {
            std::memcpy(ell, hf.data(), c->Np * sizeof(float));
        }
        c->leave();
    });
}

bdc_status bdc_logpost_trace(bdc_ctx* c, double* trace, int64_t capacity, int64_t* count) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede logpost_trace");
        const int64_t n = std::min<int64_t>(c->t, c->cfg.max_sweeps);
        if (count) *count = n;
        if (!trace) return;
        const int64_t k = std::min<int64_t>(n, capacity);
        c->enter();
        hipck(hipMemcpyAsync(trace, c->d_trace, (size_t)k * c->C * sizeof(double), hipMemcpyDeviceToHost, c->work),
              "read trace");
        c->sync();
        c->leave();
    });
}

bdc_status bdc_accept_stats(bdc_ctx* c, int64_t* accepted, int64_t* proposed) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede accept_stats");
        std::vector<unsigned long long> a(c->C);
        c->enter();
        hipck(hipMemcpyAsync(a.data(), c->d_acc, c->C * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->work),
              "read accepts");
        c->sync();
        c->leave();
        for (int i = 0; i < c->C; ++i) {
            if (accepted) accepted[i] = (int64_t)a[i];
            if (proposed) proposed[i] = c->t * c->N;
        }
    });
}

bdc_status bdc_get_state(bdc_ctx* c, void* buf, size_t* bytes) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede get_state");
        need(c, bytes != nullptr, BDC_EINVAL, "bytes is NULL");
        const size_t CN = (size_t)c->C * c->N;
        const size_t nbat = (size_t)c->max_batches * 3 * CN;
        const size_t ntr = (size_t)c->cfg.max_sweeps * c->C;
        const size_t need_b = sizeof(StateHeader) + 4 * CN * sizeof(float) + nbat * sizeof(float) +
                              ntr * sizeof(double) + c->C * sizeof(unsigned long long);
        if (!buf) { *bytes = need_b; return; }
        need(c, *bytes >= need_b, BDC_EINVAL, "state buffer too small");
        StateHeader hd{STATE_MAGIC, c->cfg.height, c->cfg.width, c->C, c->s, c->t, c->max_batches,
                       c->cfg.rhat_block, c->sub, 0, (int64_t)ntr};
        char* p = static_cast<char*>(buf);
        std::memcpy(p, &hd, sizeof(hd));
        p += sizeof(hd);
        c->enter();
        for (float* src : {c->d_rho, c->d_ls, c->d_mean, c->d_m2}) {
            hipck(hipMemcpyAsync(p, src, CN * sizeof(float), hipMemcpyDeviceToHost, c->work), "save");
            p += CN * sizeof(float);
        }
        hipck(hipMemcpyAsync(p, c->d_batch, nbat * sizeof(float), hipMemcpyDeviceToHost, c->work), "save");
        p += nbat * sizeof(float);
        hipck(hipMemcpyAsync(p, c->d_trace, ntr * sizeof(double), hipMemcpyDeviceToHost, c->work), "save");
        p += ntr * sizeof(double);
        hipck(hipMemcpyAsync(p, c->d_acc, c->C * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->work), "save");
        c->sync();
        c->leave();
        *bytes = need_b;
    });
}

bdc_status bdc_set_state(bdc_ctx* c, const void* buf, size_t bytes) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede set_state");
        need(c, buf != nullptr && bytes >= sizeof(StateHeader), BDC_EINVAL, "state buffer too small");
        StateHeader hd;
        std::memcpy(&hd, buf, sizeof(hd));
        need(c, hd.magic == STATE_MAGIC, BDC_EINVAL, "not a sampler state");
        need(c, hd.H == c->cfg.height && hd.W == c->cfg.width && hd.C == c->C && hd.s == c->s &&
                    hd.sub == c->sub && hd.nb == c->max_batches && hd.rhat_block == c->cfg.rhat_block &&
                    hd.n_trace == (int64_t)c->cfg.max_sweeps * c->C,
             BDC_EINVAL, "state was saved with a different configuration");
        const size_t CN = (size_t)c->C * c->N;
        const size_t nbat = (size_t)c->max_batches * 3 * CN;
        const size_t ntr = (size_t)c->cfg.max_sweeps * c->C;
        const size_t need_b = sizeof(StateHeader) + 4 * CN * sizeof(float) + nbat * sizeof(float) +
                              ntr * sizeof(double) + c->C * sizeof(unsigned long long);
        need(c, bytes >= need_b, BDC_EINVAL, "state buffer too small");
        const char* p = static_cast<const char*>(buf) + sizeof(hd);
        c->enter();
        for (float* dst : {c->d_rho, c->d_ls, c->d_mean, c->d_m2}) {
            hipck(hipMemcpyAsync(dst, p, CN * sizeof(float), hipMemcpyHostToDevice, c->work), "restore");
            p += CN * sizeof(float);
        }
        hipck(hipMemcpyAsync(c->d_batch, p, nbat * sizeof(float), hipMemcpyHostToDevice, c->work), "restore");
        p += nbat * sizeof(float);
        hipck(hipMemcpyAsync(c->d_trace, p, ntr * sizeof(double), hipMemcpyHostToDevice, c->work), "restore");
        p += ntr * sizeof(double);
        hipck(hipMemcpyAsync(c->d_acc, p, c->C * sizeof(unsigned long long), hipMemcpyHostToDevice, c->work),
              "restore");
        c->sync();
        set_t(c, hd.t);
        c->leave();
    });
}

bdc_status bdc_set_rho(bdc_ctx* c, const float* rho, const float* log_step, int64_t sweep, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede set_rho");
        need(c, rho && log_step, BDC_EINVAL, "rho or log_step is NULL");
        need(c, sweep >= 0, BDC_EINVAL, "sweep must be >= 0");
        const size_t CN = (size_t)c->C * c->N;
        std::vector<float> hr = fetch(c, rho, CN, on_device);
        std::vector<float> hl = fetch(c, log_step, CN, on_device);
        for (float v : hr)
            if (!(v > 0.0f) || !std::isfinite(v)) fail(BDC_EINVAL, "rho must be finite and > 0");
        check_finite(hl, "log_step");
        c->enter();
        hipck(hipMemcpyAsync(c->d_rho, hr.data(), CN * sizeof(float), hipMemcpyHostToDevice, c->work), "upload");
        hipck(hipMemcpyAsync(c->d_ls, hl.data(), CN * sizeof(float), hipMemcpyHostToDevice, c->work), "upload");
        c->sync();
        set_t(c, sweep);
        c->leave();
    });
}

bdc_status bdc_debug_run_groups(bdc_ctx* c, int32_t g0, int32_t g1, float* delta, uint8_t* accepted,
                                int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede debug_run_groups");
        const int ss = c->s * c->sub * c->sub * c->s;     // groups per block phase (colours of a block)
        const int ng = (c->sched == BDC_SCHED_CHROMATIC ? 1 : c->sched == BDC_SCHED_BLOCK9_SERIES ? 9 : 4) * ss;
        need(c, 0 <= g0 && g0 <= g1 && g1 <= ng, BDC_EINVAL, "group range out of bounds");
        const size_t CN = (size_t)c->C * c->N;
        if (!c->d_dbg_delta) {
            c->d_dbg_delta = dalloc<float>(CN);
            c->d_dbg_acc = dalloc<uint8_t>(CN);
        }
        c->enter();
        hipck(launch_fill_f32(c->d_dbg_delta, CN, NAN, c->work), "fill");
        hipck(hipMemsetAsync(c->d_dbg_acc, 0xFF, CN, c->work), "hipMemsetAsync");
        const Frame f = c->frame();
        const State S = c->state();
        hipck(launch_forward_propose(f, S, c->prior(), 1, c->work), "forward_propose");
        hipck(launch_chunk_spectra(f, S, c->work), "chunk_spectra");
        if (c->sched == BDC_SCHED_CHROMATIC) {
            for (int g = g0; g < g1; ++g)
                hipck(launch_colour_pass(f, S, c->cfg.burn_in, c->d_inv, g, c->d_dbg_delta, c->d_dbg_acc, c->work),
                      "colour_pass");
        } else {
            int g = g0;
            while (g < g1) {
                const int ph = g / ss;
                const int k0 = g % ss;
                const int k1 = std::min(ss, k0 + (g1 - g));
                if (c->sched == BDC_SCHED_BLOCK_SERIES)
                    hipck(launch_block_series(f, S, c->cfg.burn_in, c->d_inv, c->B, ph, k0, k1, c->d_dbg_delta,
                                              c->d_dbg_acc, c->work), "block_series");
                else if (c->sched == BDC_SCHED_BLOCK9_SERIES)
                    hipck(launch_wave_series(f, S, c->cfg.burn_in, c->B, ph, k0, k1, c->d_dbg_delta, c->d_dbg_acc,
                                             c->work), "wave_series");
                else
                    hipck(launch_block_phase(f, S, c->cfg.burn_in, c->d_inv, c->B, ph, k0, k1, c->d_dbg_delta,
                                             c->d_dbg_acc, c->work), "block_phase");
                g += k1 - k0;
            }
        }
        if (delta) download(c, delta, c->d_dbg_delta, CN * sizeof(float), on_device);
        if (accepted) download(c, accepted, c->d_dbg_acc, CN, on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_schedule_info(bdc_ctx* c, int32_t* n_groups, int32_t* schedule, int32_t* block) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->has_psf, BDC_ESTATE, "set_psf must precede schedule_info");
        if (n_groups)
            *n_groups = (c->sched == BDC_SCHED_CHROMATIC ? 1 : c->sched == BDC_SCHED_BLOCK9_SERIES ? 9 : 4) * c->sub *
                        c->sub * c->s * c->s;
        if (schedule) *schedule = c->sched;
        if (block) *block = c->B;
    });
}

bdc_status bdc_profile(bdc_ctx* c, int32_t enable) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        c->sync();
        c->clear_marks();
        c->profiling = enable != 0;
    });
}

bdc_status bdc_profile_read(bdc_ctx* c, double* ms, int64_t* launches, int64_t* work) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        unsigned long long w[NCOUNTERS] = {};
        c->enter();
        hipck(hipMemcpyAsync(w, c->d_ctr, sizeof(w), hipMemcpyDeviceToHost, c->work), "read counters");
        hipck(hipMemsetAsync(c->d_ctr, 0, sizeof(w), c->work), "hipMemsetAsync");
        c->sync();
        c->leave();
        double acc[3] = {0, 0, 0};
        int64_t cnt[3] = {0, 0, 0};
        for (size_t i = 1; i < c->marks.size(); ++i) {
            const int cls = c->marks[i].second;
            if (cls < 0) continue;
            float e = 0.0f;
            hipck(hipEventElapsedTime(&e, c->marks[i - 1].first, c->marks[i].first), "hipEventElapsedTime");
            acc[cls] += e;
            cnt[cls] += 1;
        }
        c->clear_marks();
        for (int k = 0; k < 3; ++k) {
            if (ms) ms[k] = acc[k];
            if (launches) launches[k] = cnt[k];
        }
        if (work)
            for (int k = 0; k < NCOUNTERS; ++k) work[k] = (int64_t)w[k];
    });
}

bdc_status bdc_philox(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* out,
                      void* hip_stream) {
    return guarded(nullptr, [&] {
        if (n < 0 || (n > 0 && (!ctr || !out))) fail(BDC_EINVAL, "bad arguments");
        if (n == 0) return;
        hipStream_t st = (hipStream_t)hip_stream;
        hipck(launch_philox(ctr, n, make_uint2(key0, key1), out, st), "philox");
        hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

// The scan of one autotuner candidate (encoding as in bdc.h).
void set_candidate(bdc_ctx* c, int b) {
    c->sched = b == 0 ? BDC_SCHED_CHROMATIC
               : b <= -1000 ? BDC_SCHED_BLOCK9_SERIES
               : b < 0      ? BDC_SCHED_BLOCK_SERIES
                            : BDC_SCHED_BLOCK;
    c->B = b <= -1000 ? -b - 1000 : b < 0 ? -b : b;
}

bdc_status bdc_autotune(bdc_ctx* c, const int32_t* blocks, int32_t n, int32_t sweeps, float* ms, int32_t* best) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede autotune");
        need(c, blocks && n > 0 && sweeps > 0, BDC_EINVAL, "need candidates and sweeps > 0");
        const int sched0 = c->sched, B0 = c->B;
        float best_ms = INFINITY;
        int best_b = 0;
        bool found = false;
        hipEvent_t e0, e1;
        hipck(hipEventCreate(&e0), "hipEventCreate");
        hipck(hipEventCreate(&e1), "hipEventCreate");
        c->enter();
        for (int i = 0; i < n; ++i) {
            const int b = blocks[i];
            float el = INFINITY;
            bool ok = b == 0 ? true
                      : b <= -1000 ? (b > -2000 && wave_series_fits(-b - 1000, c->s))
                      : b < 0 ? block_series_fits(-b, c->s)
                              : (b >= c->s - 1 && b >= 1 && b <= 4 * c->s && block_phase_lds(b, c->s) <= 64 * 1024 &&
                                 std::min(c->cfg.height, c->cfg.width) >= 2);
            // the Dirichlet-OTF prior: block-phase scan with its chunk side only
            if (c->cfg.prior_kind == BDC_PRIOR_DIRICHLET) ok = b == c->B;
            // the block-series scans take the sCMOS reading only
            if (c->cfg.camera == BDC_CAMERA_EMCCD && b < 0) ok = false;
            // a finer object lattice: the pixel-chromatic and block-phase scans
            if (c->sub > 1 && b < 0) ok = false;
            if (c->sub > 1 && b > 0) ok = b >= std::max(1, c->s - 1) && b <= 4 * c->s &&
                                      block_phase_sub_lds(b, c->s, c->sub) <= 64 * 1024;
            if (ok) {
                set_candidate(c, b);
                c->drop_graph();
                if (c->use_graph) build_graph(c);
                hipck(hipEventRecord(e0, c->work), "hipEventRecord");
                for (int k = 0; k < sweeps; ++k) {
                    if (c->graph) hipck(hipGraphLaunch(c->graph, c->work), "hipGraphLaunch");
                    else run_sweep_body(c, c->work);
                }
                hipck(hipEventRecord(e1, c->work), "hipEventRecord");
                hipck(hipEventSynchronize(e1), "hipEventSynchronize");
                hipck(hipEventElapsedTime(&el, e0, e1), "hipEventElapsedTime");
                c->t += sweeps;
                el /= sweeps;
                if (el < best_ms) { best_ms = el; best_b = b; found = true; }
            }
            if (ms) ms[i] = el;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (!found) {
            c->sched = sched0;
            c->B = B0;
        } else {
            set_candidate(c, best_b);
        }
        c->drop_graph();
        c->leave();
        if (best) *best = found ? best_b : INT32_MIN;
    });
}

bdc_status bdc_set_schedule(bdc_ctx* c, int32_t schedule, int32_t block) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->has_psf, BDC_ESTATE, "set_psf must precede set_schedule");
        need(c, schedule >= 0 && schedule <= 4 && block >= 0, BDC_EINVAL, "unknown schedule or negative block");
        const int s0 = c->cfg.schedule, b0 = c->cfg.block_size;
        c->cfg.schedule = schedule;
        c->cfg.block_size = block;
        try {
            choose_schedule(c);
        } catch (...) {
            c->cfg.schedule = s0;
            c->cfg.block_size = b0;
            choose_schedule(c);
            throw;
        }
        c->sync();
        build_dirichlet(c);
        c->drop_graph();
        c->gen++;
    });
}

bdc_status bdc_richardson_lucy(bdc_ctx* c, int32_t n_iter, float* out, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "richardson_lucy");
        need(c, c->ready, BDC_ESTATE, "init must precede richardson_lucy");
        need(c, out != nullptr && n_iter >= 0, BDC_EINVAL, "out is NULL or n_iter < 0");
        need(c, c->s <= 63, BDC_EINVAL, "PSF too large");
        c->enter();
        hipck(launch_richardson_lucy(c->frame(), n_iter, c->d_tmp, c->d_tmp2, reinterpret_cast<float*>(c->d_tmpd),
                                     c->d_lp, c->work), "richardson_lucy");
        download(c, out, c->d_tmp, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_init_rl(bdc_ctx* c, int32_t n_iter) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "init_rl");
        need(c, c->ready, BDC_ESTATE, "init must precede init_rl");
        need(c, n_iter >= 0, BDC_EINVAL, "n_iter < 0");
        c->enter();
        const Frame f = c->frame();
        hipck(launch_richardson_lucy(f, n_iter, c->d_tmp, c->d_tmp2, reinterpret_cast<float*>(c->d_tmpd), c->d_lp,
                                     c->work), "richardson_lucy");
        hipck(launch_rl_init(f, c->state(), c->d_tmp, 1e-3f, c->cfg.log_step0, c->work), "rl_init");
        const size_t CN = (size_t)c->C * c->N;
        hipck(launch_fill_f32(c->d_mean, CN, 0.0f, c->work), "fill");
        hipck(launch_fill_f32(c->d_m2, CN, 0.0f, c->work), "fill");
        hipck(hipMemsetAsync(c->d_acc, 0, c->C * sizeof(unsigned long long), c->work), "hipMemsetAsync");
        set_t(c, 0);
        c->leave();
    });
}

bdc_status bdc_set_export(bdc_ctx* c, int32_t thin, int32_t capacity) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, thin >= 0 && capacity >= 0, BDC_EINVAL, "thin and capacity must be >= 0");
        need(c, (thin == 0 || capacity == 0) || !c->ready || c->t <= c->cfg.burn_in, BDC_ESTATE,
             "the export must be set before burn-in ends");
        c->sync();
        if (c->d_samples) { (void)hipFree(c->d_samples); c->d_samples = nullptr; }
        c->exp_thin = 0;
        c->exp_cap = 0;
        if (thin > 0 && capacity > 0) {
            c->d_samples = dalloc<float>((size_t)capacity * c->C * c->N);
            c->exp_thin = thin;
            c->exp_cap = capacity;
        }
        c->drop_graph();
    });
}

bdc_status bdc_samples(bdc_ctx* c, float* out, int64_t first, int64_t count, int64_t* n_stored, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede samples");
        const int64_t ns = stored_samples(c->t, c->cfg.burn_in, c->exp_thin, c->exp_cap);
        if (n_stored) *n_stored = ns;
        if (!out || count == 0) return;
        need(c, first >= 0 && count >= 0 && first + count <= ns, BDC_EINVAL, "sample range beyond the stored samples");
        c->enter();
        const size_t CN = (size_t)c->C * c->N;
        download(c, out, c->d_samples + (size_t)first * CN, (size_t)count * CN * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_quantiles(bdc_ctx* c, const float* probs, int32_t n_probs, float* out, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede quantiles");
        need(c, probs && out && n_probs >= 1, BDC_EINVAL, "probs and out must be given, n_probs >= 1");
        for (int i = 0; i < n_probs; ++i)
            need(c, probs[i] >= 0.0f && probs[i] <= 1.0f, BDC_EINVAL, "quantile levels must lie in [0, 1]");
        const int64_t ns = stored_samples(c->t, c->cfg.burn_in, c->exp_thin, c->exp_cap);
        need(c, ns >= 1, BDC_ESTATE, "no stored samples (bdc_set_export, then post-burn-in sweeps)");
        const int64_t n = ns * c->C;
        need(c, n <= QMAX, BDC_EINVAL, "quantiles take at most 4096 values per pixel (stored samples x chains)");
        c->enter();
        if (n_probs > c->n_probs_alloc) {
            c->sync();
            if (c->d_probs) (void)hipFree(c->d_probs);
            c->d_probs = nullptr;
            c->d_probs = dalloc<float>(n_probs);
            c->n_probs_alloc = n_probs;
        }
        hipck(hipMemcpyAsync(c->d_probs, probs, n_probs * sizeof(float), hipMemcpyHostToDevice, c->work),
              "upload levels");
        float* dout = out;
        const int64_t nout = (int64_t)n_probs * c->N;
        if (!on_device) {
            if (nout > c->qout_alloc) {
                c->sync();
                if (c->d_qout) (void)hipFree(c->d_qout);
                c->d_qout = nullptr;
                c->d_qout = dalloc<float>(nout);
                c->qout_alloc = nout;
            }
            dout = c->d_qout;
        }
        hipck(launch_quantiles(c->d_samples, n, c->N, c->N, c->d_probs, n_probs, dout, c->work), "quantiles");
        if (!on_device) download(c, out, dout, nout * sizeof(float), 0);
        c->sync();
        c->leave();
    });
}

bdc_status bdc_quantiles_of(const float* samples, int64_t n, int64_t n_pix, const float* probs, int32_t n_probs,
                            float* out, void* hip_stream) {
    return guarded(nullptr, [&] {
        if (!samples || !probs || !out) fail(BDC_EINVAL, "NULL pointer");
        if (n < 1 || n > QMAX || n_pix < 1 || n_probs < 1) fail(BDC_EINVAL, "need 1 <= n <= 4096, n_pix >= 1, n_probs >= 1");
        hipStream_t st = (hipStream_t)hip_stream;
        hipck(launch_quantiles(samples, n, n_pix, n_pix, probs, n_probs, out, st), "quantiles");
        hipck(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

bdc_status bdc_cv_map(bdc_ctx* c, float* cv, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, c->ready, BDC_ESTATE, "init must precede cv_map");
        need(c, cv != nullptr, BDC_EINVAL, "cv is NULL");
        const int64_t ns = std::max<int64_t>(0, c->t - c->cfg.burn_in);
        need(c, ns >= 2, BDC_ESTATE, "fewer than 2 post-burn-in sweeps");
        c->enter();
        hipck(launch_pooled_moments(c->frame(), c->moments(), ns, -1, c->d_tmp, c->d_tmp2, c->work), "pooled moments");
        hipck(launch_cv(c->d_tmp, c->d_tmp2, c->N, c->d_tmp, c->work), "cv");
        download(c, cv, c->d_tmp, c->N * sizeof(float), on_device);
        c->sync();
        c->leave();
    });
}

const char* bdc_last_error(const bdc_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

void bdc_destroy(bdc_ctx* c) {
    if (!c) return;
    if (c->work) (void)hipStreamSynchronize(c->work);
    c->free_all();
    delete c;
}

}  // extern "C"


// ---------------------------------------------------------------------------
// Learned warm start and block independence move (bdc_unet.h)
// ---------------------------------------------------------------------------
namespace {

// Scratch of the allocation-free entry points: one array per GPU, held until
// the process ends.  Host code reaches it only through the device address
// that hipGetSymbolAddress returns for the current device (the array's name
// is a host-side stand-in, not a device address).  Calls that use it at the
// same time on one GPU race.
constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)16 << 20;      // 64 MiB
__device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

float* scratch_for_current_device() {
    int dev = 0;
    hipck(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(BDC_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        float* ptr = nullptr;
        hipck(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!ptr) fail(BDC_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

void ensure_maps(bdc_ctx* c) {
    if (!c->d_pm) {
        c->d_pm = dalloc<float>(c->N);
        c->d_ps = dalloc<float>(c->N);
        c->d_scale = dalloc<float>(1);
        c->d_bacc = dalloc<unsigned long long>(1);
        hipck(hipMemsetAsync(c->d_bacc, 0, sizeof(unsigned long long), c->work), "hipMemsetAsync");
    }
}

int n_block_colours(const bdc_ctx* c) {
    const int P = block_period(c->r);
    return P * P;
}

void block_pass(bdc_ctx* c, int64_t pass, int colour_only, float* dbg_delta, uint8_t* dbg_acc) {
    const Frame f = c->frame();
    const State S = c->state();
    hipck(launch_forward_propose(f, S, c->prior(), 0, c->work), "forward (mu refresh)");
    const int nc = n_block_colours(c);
    for (int k = 0; k < nc; ++k) {
        if (colour_only >= 0 && k != colour_only) continue;
        hipck(launch_block_colour(f, S, c->prior(), c->d_pm, c->d_ps, c->d_inv, k, (uint32_t)pass, c->block_beta,
                                  c->block_walk, c->d_bacc, dbg_delta, dbg_acc, c->work), "block_colour");
        c->block_proposed += (int64_t)block_colour_count(f, k) * c->C;
    }
}

}  // namespace

extern "C" {

bdc_status bdc_init_learned(bdc_ctx* c, bdc_unet* u) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "init_learned");
        need(c, c->ready, BDC_ESTATE, "init must precede init_learned");
        need(c, u != nullptr, BDC_EINVAL, "network is NULL");
        const int q = 1 << (bdc::unet::net_levels(u) - 1);
        const int Hp = (c->cfg.height + q - 1) / q * q, Wp = (c->cfg.width + q - 1) / q * q;
        need(c, (int64_t)Hp * Wp <= bdc::unet::net_max_pixels(u), BDC_EINVAL,
             "the padded frame exceeds the network's max_pixels");
        c->enter();
        ensure_maps(c);
        const Frame f = c->frame();
        float* x = dalloc<float>((size_t)Hp * Wp);
        try {
            hipck(launch_frame_scale(f, c->d_tmpd, c->d_scale, c->work), "frame_scale");
            hipck(launch_learned_input(f, c->d_scale, Hp, Wp, x, c->work), "learned_input");
            float* out = nullptr;
            std::string err;
            const bdc_status st = bdc::unet::net_forward_on(u, x, 1, Hp, Wp, &out, c->work, &err);
            if (st != BDC_OK) fail(st, "network forward: " + err);
            hipck(launch_learned_init(f, c->state(), out, Wp, c->d_scale, c->cfg.log_step0, c->d_pm, c->d_ps,
                                      c->work), "learned_init");
            c->sync();
        } catch (...) {
            (void)hipFree(x);
            throw;
        }
        (void)hipFree(x);
        const size_t CN = (size_t)c->C * c->N;
        hipck(launch_fill_f32(c->d_mean, CN, 0.0f, c->work), "fill");
        hipck(launch_fill_f32(c->d_m2, CN, 0.0f, c->work), "fill");
        hipck(hipMemsetAsync(c->d_acc, 0, c->C * sizeof(unsigned long long), c->work), "hipMemsetAsync");
        hipck(hipMemsetAsync(c->d_bacc, 0, sizeof(unsigned long long), c->work), "hipMemsetAsync");
        c->block_pass = 0;
        c->block_proposed = 0;
        c->has_maps = true;
        set_t(c, 0);
        c->leave();
    });
}

bdc_status bdc_set_block_proposal(bdc_ctx* c, const float* mean_log, const float* sd_log, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "set_block_proposal");
        need(c, c->has_psf && c->has_cam, BDC_ESTATE, "set_psf and set_camera_maps must precede set_block_proposal");
        need(c, mean_log && sd_log, BDC_EINVAL, "mean_log or sd_log is NULL");
        c->enter();
        std::vector<float> m = fetch(c, mean_log, (size_t)c->N, on_device);
        std::vector<float> sd = fetch(c, sd_log, (size_t)c->N, on_device);
        check_finite(m, "mean_log");
        check_finite(sd, "sd_log");
        for (float v : sd)
            if (!(v > 0.0f)) fail(BDC_EINVAL, "sd_log must be > 0");
        ensure_maps(c);
        hipck(hipMemcpyAsync(c->d_pm, m.data(), c->N * sizeof(float), hipMemcpyHostToDevice, c->work), "upload");
        hipck(hipMemcpyAsync(c->d_ps, sd.data(), c->N * sizeof(float), hipMemcpyHostToDevice, c->work), "upload");
        c->sync();
        c->has_maps = true;
        c->leave();
    });
}

bdc_status bdc_set_block_walk(bdc_ctx* c, float step) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, std::isfinite(step) && step >= 0.0f, BDC_EINVAL, "the walk step must be finite and >= 0");
        c->block_walk = step;
    });
}

bdc_status bdc_set_block_beta(bdc_ctx* c, float beta) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        need(c, beta > 0.0f && beta <= 1.0f, BDC_EINVAL, "beta must lie in (0, 1]");
        c->block_beta = beta;
    });
}

bdc_status bdc_block_move(bdc_ctx* c, int32_t n) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "block_move");
        need(c, c->ready, BDC_ESTATE, "init must precede block_move");
        need(c, c->cfg.prior_kind != BDC_PRIOR_DIRICHLET, BDC_EINVAL,
             "block moves straddle the Dirichlet-OTF prior's chunks: not available with that prior");
        need(c, c->has_maps || c->block_walk > 0.0f, BDC_ESTATE, "block proposal maps are not set");
        need(c, n >= 0, BDC_EINVAL, "n must be >= 0");
        c->enter();
        ensure_maps(c);
        for (int i = 0; i < n; ++i) {
            block_pass(c, c->block_pass, -1, nullptr, nullptr);
            c->block_pass += 1;
        }
        c->leave();
    });
}

bdc_status bdc_block_stats(bdc_ctx* c, int64_t* accepted, int64_t* proposed) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        unsigned long long a = 0;
        if (c->d_bacc) {
            hipck(hipMemcpyAsync(&a, c->d_bacc, sizeof(a), hipMemcpyDeviceToHost, c->work), "hipMemcpyAsync");
            c->sync();
        }
        if (accepted) *accepted = (int64_t)a;
        if (proposed) *proposed = c->block_proposed;
    });
}

bdc_status bdc_training_targets(bdc_ctx* c, float* x, float* target, float* scale, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "training_targets");
        need(c, c->ready, BDC_ESTATE, "init must precede training_targets");
        need(c, x && target, BDC_EINVAL, "x or target is NULL");
        const int64_t ns = std::max<int64_t>(0, c->t - c->cfg.burn_in);
        need(c, ns >= 2, BDC_ESTATE, "fewer than 2 post-burn-in sweeps");
        c->enter();
        ensure_maps(c);
        const Frame f = c->frame();
        hipck(launch_pooled_moments(f, c->moments(), ns, -1, c->d_tmp, c->d_tmp2, c->work), "pooled moments");
        hipck(launch_frame_scale(f, c->d_tmpd, c->d_scale, c->work), "frame_scale");
        float *dx = x, *dt = target;
        if (!on_device) {
            dx = c->d_pm;                     // staging: the proposal maps are not in use here
            dt = dalloc<float>((size_t)2 * c->N);
        }
        try {
            hipck(launch_training_targets(f, c->d_tmp, c->d_tmp2, c->d_scale, dx, dt, c->work), "training_targets");
            if (!on_device) {
                hipck(hipMemcpyAsync(x, dx, c->N * sizeof(float), hipMemcpyDeviceToHost, c->work), "download");
                hipck(hipMemcpyAsync(target, dt, 2 * c->N * sizeof(float), hipMemcpyDeviceToHost, c->work),
                      "download");
            }
            if (scale) hipck(hipMemcpyAsync(scale, c->d_scale, sizeof(float), hipMemcpyDeviceToHost, c->work),
                             "download");
            c->sync();
        } catch (...) {
            if (!on_device) (void)hipFree(dt);
            throw;
        }
        if (!on_device) {
            (void)hipFree(dt);
            c->has_maps = false;              // the staging overwrote the maps
        }
        c->leave();
    });
}

bdc_status bdc_training_targets_noalloc(bdc_ctx* c, float* x, float* target, float* scale, int32_t on_device) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "training_targets");
        need(c, c->ready, BDC_ESTATE, "init must precede training_targets");
        need(c, x && target, BDC_EINVAL, "x or target is NULL");
        const int64_t ns = std::max<int64_t>(0, c->t - c->cfg.burn_in);
        need(c, ns >= 2, BDC_ESTATE, "fewer than 2 post-burn-in sweeps");
        // scratch layout (floats): [0] the frame scale, [64, 64 + N) x, then 2N target
        const size_t need_f = 64 + 3 * (size_t)c->N;
        need(c, need_f <= NOALLOC_SCRATCH_FLOATS, BDC_EINVAL,
             "frame too large for the allocation-free call (at most 5592384 pixels)");
        float* ptr = scratch_for_current_device();
        float* d_sc = ptr;
        float* dx = on_device ? x : ptr + 64;
        float* dt = on_device ? target : ptr + 64 + c->N;
        c->enter();
        const Frame f = c->frame();
        hipck(launch_pooled_moments(f, c->moments(), ns, -1, c->d_tmp, c->d_tmp2, c->work), "pooled moments");
        hipck(launch_frame_scale(f, c->d_tmpd, d_sc, c->work), "frame_scale");
        hipck(launch_training_targets(f, c->d_tmp, c->d_tmp2, d_sc, dx, dt, c->work), "training_targets");
        if (!on_device) {
            hipck(hipMemcpyAsync(x, dx, c->N * sizeof(float), hipMemcpyDeviceToHost, c->work), "download");
            hipck(hipMemcpyAsync(target, dt, 2 * c->N * sizeof(float), hipMemcpyDeviceToHost, c->work), "download");
        }
        if (scale) hipck(hipMemcpyAsync(scale, d_sc, sizeof(float), hipMemcpyDeviceToHost, c->work), "download");
        c->sync();
        c->leave();
    });
}

bdc_status bdc_debug_block_colour(bdc_ctx* c, int64_t pass, int32_t colour, float* delta, uint8_t* acc,
                                  int32_t* n_blocks) {
    if (!c) return BDC_EINVAL;
    return guarded(c, [&] {
        pixel_lattice_only(c, "debug_block_colour");
        need(c, c->ready, BDC_ESTATE, "init must precede debug_block_colour");
        need(c, c->cfg.prior_kind != BDC_PRIOR_DIRICHLET, BDC_EINVAL,
             "block moves straddle the Dirichlet-OTF prior's chunks: not available with that prior");
        need(c, c->has_maps || c->block_walk > 0.0f, BDC_ESTATE, "block proposal maps are not set");
        need(c, 0 <= colour && colour < n_block_colours(c), BDC_EINVAL, "colour out of range");
        need(c, pass >= 0 && pass <= 0xFFFFFFFFll, BDC_EINVAL, "pass out of range");
        const int nb = block_colour_count(c->frame(), colour);
        if (n_blocks) *n_blocks = nb;
        c->enter();
        ensure_maps(c);
        if (!c->d_bdbg) {
            c->d_bdbg = dalloc<float>((size_t)c->C * c->N);
            c->d_bdbg_acc = dalloc<uint8_t>((size_t)c->C * c->N);
        }
        block_pass(c, pass, colour, c->d_bdbg, c->d_bdbg_acc);
        const size_t n = (size_t)c->C * nb;
        if (delta && n) hipck(hipMemcpyAsync(delta, c->d_bdbg, n * sizeof(float), hipMemcpyDeviceToHost, c->work),
                              "hipMemcpyAsync");
        if (acc && n) hipck(hipMemcpyAsync(acc, c->d_bdbg_acc, n, hipMemcpyDeviceToHost, c->work), "hipMemcpyAsync");
        c->sync();
        c->leave();
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched sweeps over several contexts (tiles)
// ---------------------------------------------------------------------------
struct bdc_batch {
    std::vector<bdc_ctx*> tiles;
    std::vector<int64_t> gens;
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<hipEvent_t> tile_ev;
    std::string err = "no error";
    TileDesc* d_tiles = nullptr;
    Item* d_items = nullptr;
    int64_t** d_tps = nullptr;
    double* d_inv = nullptr;
    int n_items = 0, cmax = 1;
    // launch segments in sweep order: one level and one kind of work each
    struct Seg { int kind, off, n; size_t lds; };
    std::vector<Seg> segs;
    hipGraphExec_t graph = nullptr;

    void free_all() {
        if (graph) (void)hipGraphExecDestroy(graph);
        void* ptrs[] = {d_tiles, d_items, d_tps, d_inv};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        for (hipEvent_t e : tile_ev) (void)hipEventDestroy(e);
        if (ev) (void)hipEventDestroy(ev);
        if (work) (void)hipStreamDestroy(work);
    }
};

namespace {

template <class F>
bdc_status bguarded(bdc_batch* b, F&& fn) {
    try {
        fn();
        if (b) b->err = "no error";
        return BDC_OK;
    } catch (const Fail& f) {
        if (b) b->err = f.msg; else g_err = f.msg;
        return f.st;
    } catch (const std::bad_alloc&) {
        if (b) b->err = "host allocation failed"; else g_err = "host allocation failed";
        return BDC_ENOMEM;
    } catch (...) {
        if (b) b->err = "unexpected internal error"; else g_err = "unexpected internal error";
        return BDC_EDEVICE;
    }
}

void batch_sweep_body(bdc_batch* b, hipStream_t st) {
    for (const bdc_batch::Seg& g : b->segs)
        hipck(launch_batch_level(g.kind, b->d_tiles, b->d_items + g.off, g.n, b->d_inv, g.lds, st), "batch level");
    hipck(launch_batch_advance(b->d_tps, (int)b->tiles.size(), st), "batch advance");
}

}  // namespace

extern "C" {

bdc_status bdc_batch_create(bdc_ctx* const* tiles, int32_t n_tiles, void* hip_stream, bdc_batch** out) {
    if (!out) { g_err = "out is NULL"; return BDC_EINVAL; }
    *out = nullptr;
    bdc_batch* b = nullptr;
    bdc_status st = bguarded(nullptr, [&] {
        if (!tiles || n_tiles < 1) fail(BDC_EINVAL, "need at least one tile");
        b = new bdc_batch();
        b->user = (hipStream_t)hip_stream;
        hipck(hipStreamCreateWithFlags(&b->work, hipStreamNonBlocking), "hipStreamCreate");
        hipck(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming), "hipEventCreate");
        std::vector<TileDesc> desc(n_tiles);
        struct WorkItem { Item it; int kind; double work; };
        std::vector<WorkItem> items;
        size_t lds_kind[BK_KINDS] = {};
        for (int i = 0; i < n_tiles; ++i) {
            bdc_ctx* c = tiles[i];
            if (!c) fail(BDC_EINVAL, "tile context is NULL");
            if (!c->ready) fail(BDC_ESTATE, "every tile must be initialised before batching");
            if (c->sched != BDC_SCHED_BLOCK && c->sched != BDC_SCHED_BLOCK_SERIES &&
                c->sched != BDC_SCHED_BLOCK9_SERIES)
                fail(BDC_EINVAL, "batched tiles must use a block-phase or block-series scan");
            if (c->cfg.prior_kind == BDC_PRIOR_DIRICHLET)
                fail(BDC_EINVAL, "batched tiles take a separable prior (the Dirichlet-OTF prior runs per context)");
            if (c->sub > 1) fail(BDC_EINVAL, "batched tiles take object lattice = pixel lattice");
            b->tiles.push_back(c);
            b->gens.push_back(c->gen);
            hipEvent_t e;
            hipck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
            b->tile_ev.push_back(e);
            TileDesc& T = desc[i];
            T.f = c->frame();
            T.S = c->state();
            T.M = c->moments();
            T.pr = c->prior();
            T.burn_in = c->cfg.burn_in;
            T.B = c->B;
            T.series = c->sched == BDC_SCHED_BLOCK9_SERIES ? 2 : c->sched == BDC_SCHED_BLOCK_SERIES ? 1 : 0;
            const int H = c->cfg.height, W = c->cfg.width, s = c->s, B = c->B, F = s * s;
            const int P = T.series == 2 ? 3 : 2;                // block phases P x P
            T.count[0] = ((H + FT_SIDE - 1) / FT_SIDE) * ((W + FT_SIDE - 1) / FT_SIDE);
            const int nby = (H + B - 1) / B, nbx = (W + B - 1) / B;
            for (int ph = 0; ph < P * P; ++ph) {
                const int py = ph / P, px = ph % P;
                T.count[1 + ph] = std::max(0, (nby - py + P - 1) / P) * std::max(0, (nbx - px + P - 1) / P);
            }
            T.count[LEV_MOMENTS] = (int)((c->N + WG - 1) / WG);
            T.count[LEV_FINALIZE] = 1;
            b->cmax = std::max(b->cmax, c->C);
            // an EMCCD tile always scans block phases (its contexts refuse the series scans)
            const bool em = c->cfg.camera == BDC_CAMERA_EMCCD;
            const int pass_kind = T.series == 2 ? (F <= 4 * 64 ? BK_WAVE4 : F <= 8 * 64 ? BK_WAVE8 : BK_WAVE16)
                                  : T.series == 1 ? BK_SERIES
                                  : em            ? BK_PHASE_EM
                                                  : BK_PHASE;
            const int moments_kind = em ? BK_MOMENTS_EM : BK_MOMENTS;
            const size_t pass_lds = T.series == 2 ? wave_series_lds(B, s)
                                    : T.series == 1 ? block_series_lds(B, s)
                                                    : block_phase_lds(B, s);
            lds_kind[BK_FORWARD] = std::max(lds_kind[BK_FORWARD], forward_lds(s));
            lds_kind[pass_kind] = std::max(lds_kind[pass_kind], pass_lds);
            for (int ch = 0; ch < c->C; ++ch) {
                for (int k = 0; k < T.count[0]; ++k)
                    items.push_back({{i, ch, 0, k}, BK_FORWARD, (double)FT_SIDE * FT_SIDE * F});
                for (int ph = 0; ph < P * P; ++ph) {
                    const int py = ph / P, px = ph % P, nbx_p = (nbx - px + P - 1) / P;
                    for (int k = 0; k < T.count[1 + ph]; ++k) {
                        const int by = py + P * (k / nbx_p), bx = px + P * (k % nbx_p);
                        const double area = (double)std::min(B, H - by * B) * std::min(B, W - bx * B);
                        items.push_back({{i, ch, 1 + ph, k}, pass_kind, area * F});
                    }
                }
                for (int k = 0; k < T.count[LEV_MOMENTS]; ++k)
                    items.push_back({{i, ch, LEV_MOMENTS, k}, moments_kind, (double)WG});
                items.push_back({{i, ch, LEV_FINALIZE, 0}, BK_FINALIZE, 1.0});
            }
        }
        // level-major order (every dependency precedes its dependants), then by kind,
        // longest first within a segment
        std::stable_sort(items.begin(), items.end(), [](const WorkItem& x, const WorkItem& y) {
            if (x.it.level != y.it.level) return x.it.level < y.it.level;
            if (x.kind != y.kind) return x.kind < y.kind;
            return x.work > y.work;
        });
        std::vector<Item> flat(items.size());
        for (size_t k = 0; k < items.size(); ++k) {
            flat[k] = items[k].it;
            if (k == 0 || items[k].it.level != items[k - 1].it.level || items[k].kind != items[k - 1].kind)
                b->segs.push_back({items[k].kind, (int)k, 0, lds_kind[items[k].kind]});
            b->segs.back().n++;
        }
        for (size_t k = 0; k < BK_KINDS; ++k)
            if (lds_kind[k] > 64 * 1024) fail(BDC_EINVAL, "a tile needs more than 64 KiB of LDS");
        b->n_items = (int)flat.size();
        b->d_tiles = dalloc<TileDesc>(n_tiles);
        b->d_items = dalloc<Item>(flat.size());
        b->d_tps = dalloc<int64_t*>(n_tiles);
        std::vector<int64_t*> tps(n_tiles);
        for (int i = 0; i < n_tiles; ++i) tps[i] = b->tiles[i]->d_t;
        std::vector<double> inv(INV_TABLE);
        inv[0] = 0.0;
        for (int i = 1; i < INV_TABLE; ++i) inv[i] = 1.0 / (double)i;
        b->d_inv = dalloc<double>(INV_TABLE);
        hipck(hipMemcpy(b->d_tiles, desc.data(), n_tiles * sizeof(TileDesc), hipMemcpyHostToDevice), "upload");
        hipck(hipMemcpy(b->d_items, flat.data(), flat.size() * sizeof(Item), hipMemcpyHostToDevice), "upload");
        hipck(hipMemcpy(b->d_tps, tps.data(), n_tiles * sizeof(int64_t*), hipMemcpyHostToDevice), "upload");
        hipck(hipMemcpy(b->d_inv, inv.data(), INV_TABLE * sizeof(double), hipMemcpyHostToDevice), "upload");
    });
    if (st != BDC_OK) {
        if (b) { b->free_all(); delete b; }
        return st;
    }
    *out = b;
    return BDC_OK;
}

bdc_status bdc_batch_sweep(bdc_batch* b, int32_t n) {
    if (!b) return BDC_EINVAL;
    return bguarded(b, [&] {
        if (n < 0) fail(BDC_EINVAL, "n must be >= 0");
        for (size_t i = 0; i < b->tiles.size(); ++i)
            if (b->tiles[i]->gen != b->gens[i] || !b->tiles[i]->ready)
                fail(BDC_ESTATE, "a tile's PSF or camera changed (or it lost its state): recreate the batch");
        if (n == 0) return;
        // order after the caller's stream and after every tile's own work
        hipck(hipEventRecord(b->ev, b->user), "hipEventRecord");
        hipck(hipStreamWaitEvent(b->work, b->ev, 0), "hipStreamWaitEvent");
        for (size_t i = 0; i < b->tiles.size(); ++i) {
            hipck(hipEventRecord(b->tile_ev[i], b->tiles[i]->work), "hipEventRecord");
            hipck(hipStreamWaitEvent(b->work, b->tile_ev[i], 0), "hipStreamWaitEvent");
        }
        if (!b->graph) {
            hipGraph_t g = nullptr;
            hipck(hipStreamBeginCapture(b->work, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            try {
                batch_sweep_body(b, b->work);
            } catch (...) {
                (void)hipStreamEndCapture(b->work, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            hipck(hipStreamEndCapture(b->work, &g), "hipStreamEndCapture");
            hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            hipck(e, "hipGraphInstantiate");
        }
        for (int k = 0; k < n; ++k) hipck(hipGraphLaunch(b->graph, b->work), "hipGraphLaunch");
        for (bdc_ctx* c : b->tiles) c->t += n;
        hipck(hipEventRecord(b->ev, b->work), "hipEventRecord");
        hipck(hipStreamWaitEvent(b->user, b->ev, 0), "hipStreamWaitEvent");
        for (bdc_ctx* c : b->tiles) hipck(hipStreamWaitEvent(c->work, b->ev, 0), "hipStreamWaitEvent");
    });
}

bdc_status bdc_batch_check(bdc_batch* b) {
    if (!b) return BDC_EINVAL;
    return bguarded(b, [&] { hipck(hipStreamSynchronize(b->work), "hipStreamSynchronize"); });
}

bdc_status bdc_batch_info(bdc_batch* b, int64_t* n_items, int32_t* grid, int32_t* lds_bytes) {
    if (!b) return BDC_EINVAL;
    if (n_items) *n_items = b->n_items;
    if (grid) {
        int mx = 0;
        for (const bdc_batch::Seg& g : b->segs) mx = std::max(mx, g.n);
        *grid = mx;
    }
    if (lds_bytes) {
        size_t mx = 0;
        for (const bdc_batch::Seg& g : b->segs) mx = std::max(mx, g.lds);
        *lds_bytes = (int32_t)mx;
    }
    return BDC_OK;
}

const char* bdc_batch_last_error(const bdc_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

void bdc_batch_destroy(bdc_batch* b) {
    if (!b) return;
    if (b->work) (void)hipStreamSynchronize(b->work);
    b->free_all();
    delete b;
}

}  // extern "C"
