// unet_runtime.cpp -- host side of the U-Net behind include/bdc_unet.h: the
// parameter layout, the activation and gradient buffers, and the launch
// sequences of the forward pass, the backward pass and the Adam step.
#include "../../include/bdc_unet.h"
#include "unet.h"
#include "unet_net.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace bdc::unet;

namespace {

thread_local std::string g_uerr = "no error";

struct UFail {
    bdc_status st;
    std::string msg;
};

[[noreturn]] void ufail(bdc_status st, const std::string& msg) { throw UFail{st, msg}; }

void uck(hipError_t e, const char* what) {
    if (e != hipSuccess) ufail(BDC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T* ualloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ufail(BDC_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return static_cast<T*>(p);
}

enum Kind { CONV3, UP, HEAD };

struct Layer {
    Kind kind;
    int cin, cout;
    int64_t w, b;            // offsets in the FP32 parameters
    int64_t wf, wd;          // offsets of the BF16 forward / dgrad operand copies (wd = -1: none)
};

constexpr int MAX_SPLITS = 512;                // enough for ~1000 workgroups on the shallowest layers
constexpr int64_t PART_FLOATS = 1 << 24;   // split-K partial buffer (64 MiB)
constexpr int COLSUM_WG = 1024;

}  // namespace

struct bdc_unet {
    bdc_unet_config cfg{};
    std::string err = "no error";
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;

    int L = 0;
    std::vector<int> ch;           // channels per level
    std::vector<Layer> layers;
    int64_t n_params = 0, n_wbf = 0;
    // indices into layers
    std::vector<int> enc1, enc2, up, dec1, dec2;
    int bott1 = -1, bott2 = -1, head = -1;

    float* params = nullptr;       // FP32 master
    float* grads = nullptr;        // n_params + 1 (loss sum last)
    float *m1 = nullptr, *m2 = nullptr;
    uint16_t* wbf = nullptr;
    int64_t step = 0;

    // activations: per level l < L-1
    uint16_t* x0 = nullptr;
    std::vector<uint16_t*> ea, cat, pool, da, db;
    uint16_t *ba = nullptr, *bb = nullptr;
    std::vector<uint16_t*> g_ea, g_cat, g_pool, g_da, g_db;
    uint16_t *g_ba = nullptr, *g_bb = nullptr;
    float* out = nullptr;          // [max_pixels][2]
    float* part = nullptr;         // split-K partials
    float* cpart = nullptr;        // column-sum / head partials
    float* tmp_in = nullptr;       // [max_pixels] staging of host inputs
    float* tmp_tgt = nullptr;      // [max_pixels][2]
    std::vector<void*> owned;

    template <class T>
    T* own(size_t n) {
        T* p = ualloc<T>(n);
        owned.push_back(p);
        return p;
    }

    void enter() {
        uck(hipEventRecord(ev_in, user), "hipEventRecord");
        uck(hipStreamWaitEvent(work, ev_in, 0), "hipStreamWaitEvent");
    }
    void leave() {
        uck(hipEventRecord(ev_out, work), "hipEventRecord");
        uck(hipStreamWaitEvent(user, ev_out, 0), "hipStreamWaitEvent");
    }
    ~bdc_unet() {
        for (void* p : owned) (void)hipFree(p);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (work) (void)hipStreamDestroy(work);
    }

    int add(Kind k, int cin, int cout) {
        Layer l{k, cin, cout, n_params, 0, n_wbf, -1};
        if (k == CONV3) {
            l.b = l.w + (int64_t)cout * 9 * cin;
            n_params = l.b + cout;
            const int kp = cin == 1 ? 16 : 9 * cin;
            n_wbf += (int64_t)cout * kp;
            if (cin != 1) { l.wd = n_wbf; n_wbf += (int64_t)cout * 9 * cin; }
        } else if (k == UP) {
            l.b = l.w + (int64_t)4 * cout * cin;
            n_params = l.b + cout;
            n_wbf += (int64_t)4 * cout * cin;
            l.wd = n_wbf;
            n_wbf += (int64_t)4 * cout * cin;
        } else {
            l.b = l.w + 2 * cin;
            n_params = l.b + 2;
            l.wf = -1;
        }
        layers.push_back(l);
        return (int)layers.size() - 1;
    }

    void build_layers() {
        ch.resize(L);
        for (int l = 0; l < L; ++l) ch[l] = cfg.base_channels << l;
        int cin = 1;
        for (int l = 0; l < L - 1; ++l) {
            enc1.push_back(add(CONV3, cin, ch[l]));
            enc2.push_back(add(CONV3, ch[l], ch[l]));
            cin = ch[l];
        }
        bott1 = add(CONV3, ch[L - 2], ch[L - 1]);
        bott2 = add(CONV3, ch[L - 1], ch[L - 1]);
        up.assign(L - 1, -1); dec1.assign(L - 1, -1); dec2.assign(L - 1, -1);
        for (int l = L - 2; l >= 0; --l) {
            up[l] = add(UP, ch[l + 1], ch[l]);
            dec1[l] = add(CONV3, 2 * ch[l], ch[l]);
            dec2[l] = add(CONV3, ch[l], ch[l]);
        }
        head = add(HEAD, ch[0], 2);
    }

    void alloc() {
        const int64_t P = cfg.max_pixels;
        params = own<float>(n_params);
        wbf = own<uint16_t>(n_wbf);
        uck(hipMemset(params, 0, n_params * sizeof(float)), "hipMemset");
        uck(hipMemset(wbf, 0, n_wbf * sizeof(uint16_t)), "hipMemset");
        x0 = own<uint16_t>(P);
        out = own<float>(2 * P);
        tmp_in = own<float>(P);
        ea.resize(L - 1); cat.resize(L - 1); pool.resize(L - 1); da.resize(L - 1); db.resize(L - 1);
        for (int l = 0; l < L - 1; ++l) {
            const int64_t Pl = P >> (2 * l);
            ea[l] = own<uint16_t>(Pl * ch[l]);
            cat[l] = own<uint16_t>(Pl * 2 * ch[l]);
            pool[l] = own<uint16_t>((Pl >> 2) * ch[l]);
            da[l] = own<uint16_t>(Pl * ch[l]);
            db[l] = own<uint16_t>(Pl * ch[l]);
        }
        const int64_t Pb = P >> (2 * (L - 1));
        ba = own<uint16_t>(Pb * ch[L - 1]);
        bb = own<uint16_t>(Pb * ch[L - 1]);
        const int64_t hrows = head_partial_rows(P);
        cpart = own<float>(std::max<int64_t>((int64_t)COLSUM_WG * 256, hrows * (2 * ch[0] + 3)));
        if (!cfg.training) return;
        grads = own<float>(n_params + 1);
        m1 = own<float>(n_params);
        m2 = own<float>(n_params);
        uck(hipMemset(m1, 0, n_params * sizeof(float)), "hipMemset");
        uck(hipMemset(m2, 0, n_params * sizeof(float)), "hipMemset");
        tmp_tgt = own<float>(2 * P);
        part = own<float>(PART_FLOATS);
        g_ea.resize(L - 1); g_cat.resize(L - 1); g_pool.resize(L - 1); g_da.resize(L - 1); g_db.resize(L - 1);
        for (int l = 0; l < L - 1; ++l) {
            const int64_t Pl = P >> (2 * l);
            g_ea[l] = own<uint16_t>(Pl * ch[l]);
            g_cat[l] = own<uint16_t>(Pl * 2 * ch[l]);
            g_pool[l] = own<uint16_t>((Pl >> 2) * ch[l]);
            g_da[l] = own<uint16_t>(Pl * ch[l]);
            g_db[l] = own<uint16_t>(Pl * ch[l]);
        }
        g_ba = own<uint16_t>(Pb * ch[L - 1]);
        g_bb = own<uint16_t>(Pb * ch[L - 1]);
    }

    void refresh_weights(hipStream_t st) {
        for (const Layer& l : layers) {
            if (l.kind == CONV3)
                uck(weights_conv3(params + l.w, l.cout, l.cin, wbf + l.wf, l.wd >= 0 ? wbf + l.wd : nullptr, st),
                    "weights_conv3");
            else if (l.kind == UP)
                uck(weights_up(params + l.w, l.cout, l.cin, wbf + l.wf, wbf + l.wd, st), "weights_up");
        }
    }

    // --- tensor views for a batch of B x H x W ------------------------------
    int H = 0, W = 0, Bn = 0;
    int64_t Pl(int l) const { return (int64_t)Bn * (H >> l) * (W >> l); }
    Tens T(uint16_t* p, int C, int ld, int off, int l) const { return Tens{p, C, ld, off, H >> l, W >> l}; }
    Tens in_t(int l) const { return l == 0 ? T(x0, 1, 1, 0, 0) : T(pool[l - 1], ch[l - 1], ch[l - 1], 0, l); }
    Tens skip_t(int l) const { return T(cat[l], ch[l], 2 * ch[l], ch[l], l); }
    Tens gskip_t(int l) const { return T(g_cat[l], ch[l], 2 * ch[l], ch[l], l); }
    Tens up_t(int l) const { return T(cat[l], ch[l], 2 * ch[l], 0, l); }
    Tens gup_t(int l) const { return T(g_cat[l], ch[l], 2 * ch[l], 0, l); }
    Tens cat_t(int l) const { return T(cat[l], 2 * ch[l], 2 * ch[l], 0, l); }
    Tens gcat_t(int l) const { return T(g_cat[l], 2 * ch[l], 2 * ch[l], 0, l); }
    Tens ea_t(int l) const { return T(ea[l], ch[l], ch[l], 0, l); }
    Tens gea_t(int l) const { return T(g_ea[l], ch[l], ch[l], 0, l); }
    Tens da_t(int l) const { return T(da[l], ch[l], ch[l], 0, l); }
    Tens gda_t(int l) const { return T(g_da[l], ch[l], ch[l], 0, l); }
    Tens db_t(int l) const { return T(db[l], ch[l], ch[l], 0, l); }
    Tens gdb_t(int l) const { return T(g_db[l], ch[l], ch[l], 0, l); }
    Tens ba_t() const { return T(ba, ch[L - 1], ch[L - 1], 0, L - 1); }
    Tens bb_t() const { return T(bb, ch[L - 1], ch[L - 1], 0, L - 1); }
    Tens gba_t() const { return T(g_ba, ch[L - 1], ch[L - 1], 0, L - 1); }
    Tens gbb_t() const { return T(g_bb, ch[L - 1], ch[L - 1], 0, L - 1); }
    Tens gpool_t(int l) const { return T(g_pool[l], ch[l], ch[l], 0, l + 1); }

    void check_shape(int B, int h, int w) {
        const int q = 1 << (L - 1);
        if (B < 1 || h < q || w < q || h % q || w % q)
            ufail(BDC_EINVAL, "batch >= 1 and height, width multiples of " + std::to_string(q) + " are required");
        if ((int64_t)B * h * w > cfg.max_pixels) ufail(BDC_EINVAL, "batch * height * width exceeds max_pixels");
        Bn = B; H = h; W = w;
    }

    const float* wb(int li) const { return params + layers[li].b; }
    const uint16_t* wf(int li) const { return wbf + layers[li].wf; }
    const uint16_t* wd(int li) const { return wbf + layers[li].wd; }

    // x: device [B][H][W]; result in `out`
    void forward(const float* x, hipStream_t st) {
        uck(to_bf16(x, Pl(0), x0, st), "to_bf16");
        for (int l = 0; l < L - 1; ++l) {
            uck(conv3_fwd(in_t(l), wf(enc1[l]), wb(enc1[l]), 1, ea_t(l), Pl(l), st), "conv3_fwd");
            uck(conv3_fwd(ea_t(l), wf(enc2[l]), wb(enc2[l]), 1, skip_t(l), Pl(l), st), "conv3_fwd");
            uck(maxpool(skip_t(l), in_t(l + 1), Pl(l + 1), st), "maxpool");
        }
        uck(conv3_fwd(in_t(L - 1), wf(bott1), wb(bott1), 1, ba_t(), Pl(L - 1), st), "conv3_fwd");
        uck(conv3_fwd(ba_t(), wf(bott2), wb(bott2), 1, bb_t(), Pl(L - 1), st), "conv3_fwd");
        for (int l = L - 2; l >= 0; --l) {
            const Tens src = l == L - 2 ? bb_t() : db_t(l + 1);
            uck(up_fwd(src, wf(up[l]), wb(up[l]), up_t(l), Pl(l + 1), H >> (l + 1), W >> (l + 1), st), "up_fwd");
            uck(conv3_fwd(cat_t(l), wf(dec1[l]), wb(dec1[l]), 1, da_t(l), Pl(l), st), "conv3_fwd");
            uck(conv3_fwd(da_t(l), wf(dec2[l]), wb(dec2[l]), 1, db_t(l), Pl(l), st), "conv3_fwd");
        }
        const Layer& h = layers[head];
        uck(bdc::unet::head(db_t(0), params + h.w, params + h.b, Pl(0), out, nullptr, nullptr, cpart, nullptr, st),
            "head");
    }

    void conv_back(int li, const Tens& x, const Tens& g, const Tens* gx, const Tens* mask, int l, hipStream_t st) {
        const Layer& ly = layers[li];
        const int64_t splits_cap = std::max<int64_t>(1, std::min<int64_t>(MAX_SPLITS,
                                                     PART_FLOATS / ((int64_t)ly.cout * 9 * ly.cin)));
        uck(conv3_wgrad(x, g, part, (int)splits_cap, grads + ly.w, Pl(l), st), "conv3_wgrad");
        uck(bias_grad(g, Pl(l), cpart, COLSUM_WG, grads + ly.b, st), "bias_grad");
        if (gx) uck(conv3_dgrad(g, wd(li), *gx, mask, Pl(l), st), "conv3_dgrad");
    }

    // forward + backward into `grads` (loss sum at grads[n_params])
    void backward(const float* x, const float* target, hipStream_t st) {
        forward(x, st);
        const Layer& h = layers[head];
        uck(bdc::unet::head(db_t(0), params + h.w, params + h.b, Pl(0), out, target, g_db[0], cpart,
                            grads + h.w, st), "head");
        for (int l = 0; l < L - 1; ++l) {
            const Tens mda = da_t(l);
            const Tens gda = gda_t(l), gcat = gcat_t(l);
            conv_back(dec2[l], da_t(l), gdb_t(l), &gda, &mda, l, st);
            conv_back(dec1[l], cat_t(l), gda_t(l), &gcat, nullptr, l, st);
            const Tens src = l == L - 2 ? bb_t() : db_t(l + 1);
            const Tens gsrc = l == L - 2 ? gbb_t() : gdb_t(l + 1);
            const Layer& ul = layers[up[l]];
            const int64_t splits_cap = std::max<int64_t>(1, std::min<int64_t>(MAX_SPLITS,
                                                         PART_FLOATS / ((int64_t)ul.cout * ul.cin)));
            uck(up_wgrad(src, gup_t(l), part, (int)splits_cap, grads + ul.w, Pl(l + 1), H >> (l + 1),
                         W >> (l + 1), st), "up_wgrad");
            uck(bias_grad(gup_t(l), Pl(l), cpart, COLSUM_WG, grads + ul.b, st), "bias_grad");
            uck(up_dgrad(gup_t(l), wd(up[l]), gsrc, &src, Pl(l + 1), H >> (l + 1), W >> (l + 1), st), "up_dgrad");
        }
        {
            const Tens mba = ba_t(), gba = gba_t(), gp = gpool_t(L - 2);
            conv_back(bott2, ba_t(), gbb_t(), &gba, &mba, L - 1, st);
            conv_back(bott1, in_t(L - 1), gba_t(), &gp, nullptr, L - 1, st);
        }
        for (int l = L - 2; l >= 0; --l) {
            uck(maxpool_bwd(skip_t(l), gskip_t(l), gpool_t(l), Pl(l + 1), st), "maxpool_bwd");
            const Tens mea = ea_t(l), gea = gea_t(l);
            conv_back(enc2[l], ea_t(l), gskip_t(l), &gea, &mea, l, st);
            if (l > 0) {
                const Tens gp = gpool_t(l - 1);
                conv_back(enc1[l], in_t(l), gea_t(l), &gp, nullptr, l, st);
            } else {
                conv_back(enc1[l], in_t(l), gea_t(l), nullptr, nullptr, l, st);
            }
        }
    }

    double flops(int B, int h, int w) const {
        double f = 0.0;
        auto P = [&](int l) { return (double)B * (h >> l) * (w >> l); };
        for (int l = 0; l < L - 1; ++l) {
            f += 2.0 * 9 * layers[enc1[l]].cin * ch[l] * P(l) + 2.0 * 9 * ch[l] * ch[l] * P(l);
            f += 2.0 * 4 * ch[l + 1] * ch[l] * P(l + 1);                    // transposed conv
            f += 2.0 * 9 * 2 * ch[l] * ch[l] * P(l) + 2.0 * 9 * ch[l] * ch[l] * P(l);
        }
        f += 2.0 * 9 * ch[L - 2] * ch[L - 1] * P(L - 1) + 2.0 * 9 * ch[L - 1] * ch[L - 1] * P(L - 1);
        f += 2.0 * 2 * ch[0] * P(0);
        return f;
    }
};

namespace {

template <class F>
bdc_status uguarded(bdc_unet* u, F&& fn) {
    try {
        fn();
        if (u) u->err = "no error";
        return BDC_OK;
    } catch (const UFail& f) {
        if (u) u->err = f.msg; else g_uerr = f.msg;
        return f.st;
    } catch (const std::bad_alloc&) {
        if (u) u->err = "host allocation failed"; else g_uerr = "host allocation failed";
        return BDC_ENOMEM;
    } catch (...) {
        if (u) u->err = "unexpected internal error"; else g_uerr = "unexpected internal error";
        return BDC_EDEVICE;
    }
}

// Device pointer for an input that may live on the host.
const float* stage(bdc_unet* u, const float* p, int64_t n, int on_device, float* dst) {
    if (on_device) return p;
    uck(hipMemcpyAsync(dst, p, n * sizeof(float), hipMemcpyHostToDevice, u->work), "hipMemcpyAsync");
    return dst;
}

void check_finite_host(const float* p, int64_t n, const char* what) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) ufail(BDC_ENOTFINITE, std::string(what) + " has a non-finite value");
}

}  // namespace

// ---- internal interface for the sampler runtime ----------------------------
namespace bdc {
namespace unet {

bdc_status net_forward_on(bdc_unet* u, const float* x_dev, int B, int h, int w, float** out_dev, hipStream_t st,
                          std::string* err) {
    const bdc_status s = uguarded(u, [&] {
        u->check_shape(B, h, w);
        u->forward(x_dev, st);
        *out_dev = u->out;
    });
    if (s != BDC_OK && err) *err = u->err;
    return s;
}

int net_levels(const bdc_unet* u) { return u->L; }
int64_t net_max_pixels(const bdc_unet* u) { return u->cfg.max_pixels; }

}  // namespace unet
}  // namespace bdc

extern "C" {

bdc_status bdc_unet_create(const bdc_unet_config* cfg, void* hip_stream, bdc_unet** out) {
    if (!out) { g_uerr = "out is NULL"; return BDC_EINVAL; }
    *out = nullptr;
    bdc_unet* u = nullptr;
    const bdc_status st = uguarded(nullptr, [&] {
        if (!cfg) ufail(BDC_EINVAL, "cfg is NULL");
        if (cfg->levels < 2 || cfg->levels > 6) ufail(BDC_EINVAL, "levels must be in 2..6");
        const int b = cfg->base_channels;
        if (b != 8 && b != 16 && b != 32 && b != 64) ufail(BDC_EINVAL, "base_channels must be 8, 16, 32 or 64");
        if ((int64_t)b << (cfg->levels - 1) > 256) ufail(BDC_EINVAL, "the deepest level exceeds 256 channels");
        const int64_t q = (int64_t)1 << (2 * (cfg->levels - 1));
        if (cfg->max_pixels < q) ufail(BDC_EINVAL, "max_pixels is below one deepest-level pixel");
        u = new bdc_unet();
        u->cfg = *cfg;
        u->L = cfg->levels;
        u->user = (hipStream_t)hip_stream;
        uck(hipStreamCreateWithFlags(&u->work, hipStreamNonBlocking), "hipStreamCreate");
        uck(hipEventCreateWithFlags(&u->ev_in, hipEventDisableTiming), "hipEventCreate");
        uck(hipEventCreateWithFlags(&u->ev_out, hipEventDisableTiming), "hipEventCreate");
        u->build_layers();
        u->alloc();
        uck(hipDeviceSynchronize(), "hipDeviceSynchronize");
    });
    if (st != BDC_OK) {
        delete u;
        return st;
    }
    *out = u;
    return BDC_OK;
}

bdc_status bdc_unet_param_count(const bdc_unet* u, int64_t* n) {
    if (!u || !n) { g_uerr = "NULL argument"; return BDC_EINVAL; }
    *n = u->n_params;
    return BDC_OK;
}

bdc_status bdc_unet_flops(const bdc_unet* u, int32_t batch, int32_t height, int32_t width, double* flops) {
    if (!u || !flops) { g_uerr = "NULL argument"; return BDC_EINVAL; }
    *flops = u->flops(batch, height, width);
    return BDC_OK;
}

bdc_status bdc_unet_set_params(bdc_unet* u, const float* params, int32_t on_device) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!params) ufail(BDC_EINVAL, "params is NULL");
        std::vector<float> h(u->n_params);
        if (on_device) uck(hipMemcpy(h.data(), params, h.size() * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
        else std::memcpy(h.data(), params, h.size() * sizeof(float));
        check_finite_host(h.data(), u->n_params, "params");
        u->enter();
        uck(hipMemcpyAsync(u->params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, u->work),
            "hipMemcpyAsync");
        u->refresh_weights(u->work);
        uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
        u->leave();
    });
}

bdc_status bdc_unet_get_params(bdc_unet* u, float* params, int32_t on_device) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!params) ufail(BDC_EINVAL, "params is NULL");
        u->enter();
        uck(hipMemcpyAsync(params, u->params, u->n_params * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, u->work), "hipMemcpyAsync");
        uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
        u->leave();
    });
}

bdc_status bdc_unet_forward(bdc_unet* u, const float* x, int32_t batch, int32_t height, int32_t width, float* out,
                            int32_t on_device) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!x || !out) ufail(BDC_EINVAL, "x or out is NULL");
        u->check_shape(batch, height, width);
        const int64_t P = (int64_t)batch * height * width;
        u->enter();
        const float* xd = stage(u, x, P, on_device, u->tmp_in);
        u->forward(xd, u->work);
        uck(hipMemcpyAsync(out, u->out, 2 * P * sizeof(float),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, u->work), "hipMemcpyAsync");
        if (!on_device) uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
        u->leave();
    });
}

bdc_status bdc_unet_gradients(bdc_unet* u, const float* x, const float* target, int32_t batch, int32_t height,
                              int32_t width, float* grads, float* loss, int32_t on_device) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!u->cfg.training) ufail(BDC_ESTATE, "network was created without training buffers");
        if (!x || !target) ufail(BDC_EINVAL, "x or target is NULL");
        u->check_shape(batch, height, width);
        const int64_t P = (int64_t)batch * height * width;
        u->enter();
        const float* xd = stage(u, x, P, on_device, u->tmp_in);
        const float* td = stage(u, target, 2 * P, on_device, u->tmp_tgt);
        u->backward(xd, td, u->work);
        if (grads)
            uck(hipMemcpyAsync(grads, u->grads, u->n_params * sizeof(float),
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, u->work),
                "hipMemcpyAsync");
        if (loss) {
            float s = 0.0f;
            uck(hipMemcpyAsync(&s, u->grads + u->n_params, sizeof(float), hipMemcpyDeviceToHost, u->work),
                "hipMemcpyAsync");
            uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
            *loss = s / (float)P;
        } else if (!on_device) {
            uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
        }
        u->leave();
    });
}

bdc_status bdc_unet_train_step(bdc_unet* u, const float* x, const float* target, int32_t batch, int32_t height,
                               int32_t width, float lr, float* loss, int32_t on_device) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!u->cfg.training) ufail(BDC_ESTATE, "network was created without training buffers");
        if (!x || !target) ufail(BDC_EINVAL, "x or target is NULL");
        if (!(lr > 0.0f) || !std::isfinite(lr)) ufail(BDC_EINVAL, "lr must be positive and finite");
        u->check_shape(batch, height, width);
        const int64_t P = (int64_t)batch * height * width;
        u->enter();
        const float* xd = stage(u, x, P, on_device, u->tmp_in);
        const float* td = stage(u, target, 2 * P, on_device, u->tmp_tgt);
        u->backward(xd, td, u->work);
        u->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = (float)(1.0 - std::pow((double)b1, (double)u->step));
        const float c2 = (float)(1.0 - std::pow((double)b2, (double)u->step));
        uck(adam(u->params, u->m1, u->m2, u->grads, u->n_params, lr, b1, b2, 1e-8f, c1, c2, u->work), "adam");
        u->refresh_weights(u->work);
        if (loss) {
            float s = 0.0f;
            uck(hipMemcpyAsync(&s, u->grads + u->n_params, sizeof(float), hipMemcpyDeviceToHost, u->work),
                "hipMemcpyAsync");
            uck(hipStreamSynchronize(u->work), "hipStreamSynchronize");
            *loss = s / (float)P;
        }
        u->leave();
    });
}

bdc_status bdc_unet_reset_optimizer(bdc_unet* u) {
    if (!u) { g_uerr = "u is NULL"; return BDC_EINVAL; }
    return uguarded(u, [&] {
        if (!u->cfg.training) ufail(BDC_ESTATE, "network was created without training buffers");
        u->enter();
        uck(hipMemsetAsync(u->m1, 0, u->n_params * sizeof(float), u->work), "hipMemsetAsync");
        uck(hipMemsetAsync(u->m2, 0, u->n_params * sizeof(float), u->work), "hipMemsetAsync");
        u->step = 0;
        u->leave();
    });
}

bdc_status bdc_debug_gemm_bf16(const uint16_t* a, const uint16_t* b, float* c, int64_t m, int32_t n, int32_t k) {
    uint16_t *da = nullptr, *db = nullptr;
    float* dc = nullptr;
    const bdc_status st = uguarded(nullptr, [&] {
        if (!a || !b || !c) ufail(BDC_EINVAL, "NULL argument");
        if (m < 1 || n < 1 || k < 8 || k % 8) ufail(BDC_EINVAL, "m, n >= 1 and k a positive multiple of 8 are required");
        da = ualloc<uint16_t>((size_t)m * k);
        db = ualloc<uint16_t>((size_t)n * k);
        dc = ualloc<float>((size_t)m * n);
        uck(hipMemcpy(da, a, (size_t)m * k * 2, hipMemcpyHostToDevice), "hipMemcpy");
        uck(hipMemcpy(db, b, (size_t)n * k * 2, hipMemcpyHostToDevice), "hipMemcpy");
        uck(gemm_nt(da, db, dc, m, n, k, nullptr), "gemm_nt");
        uck(hipMemcpy(c, dc, (size_t)m * n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    });
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (dc) (void)hipFree(dc);
    return st;
}

const char* bdc_unet_last_error(const bdc_unet* u) { return u ? u->err.c_str() : g_uerr.c_str(); }

void bdc_unet_destroy(bdc_unet* u) {
    if (!u) return;
    if (u->work) (void)hipStreamSynchronize(u->work);
    delete u;
}

}  // extern "C"
