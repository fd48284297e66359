// C ABI of the warm-start network (include/lbm_nn.h): layer table,
// workspace layout and the order of kernel launches for the forward pass,
// the backward pass and the Adam update.
#include "../../include/lbm_nn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "lbm_handle.hpp"
#include "nn_internal.hpp"

using namespace lbmnn;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Layer table: input x1 (c1 channels on the layer's level), optional x2
// (c2 channels one level coarser, upsampled), output channels, kernel taps,
// level (0 = G, 1 = G/2, ...).
struct LayerDef {
    const char* name;
    int c1, c2, cout, taps, level, relu;
};
constexpr int kLayers = 16;
static_assert(kLayers <= kMaxPackLayers, "one packing launch covers every layer");
constexpr LayerDef kDefs[kLayers] = {
    {"enc1a", 4, 0, 16, 27, 0, 1},    {"enc1b", 16, 0, 16, 27, 0, 1},
    {"enc2a", 16, 0, 32, 27, 1, 1},   {"enc2b", 32, 0, 32, 27, 1, 1},
    {"enc3a", 32, 0, 64, 27, 2, 1},   {"enc3b", 64, 0, 64, 27, 2, 1},
    {"bota", 64, 0, 128, 27, 3, 1},   {"botb", 128, 0, 128, 27, 3, 1},
    {"botc", 128, 0, 128, 27, 3, 1},  {"dec3a", 64, 128, 64, 27, 2, 1},
    {"dec3b", 64, 0, 64, 27, 2, 1},   {"dec2a", 32, 64, 32, 27, 1, 1},
    {"dec2b", 32, 0, 32, 27, 1, 1},   {"dec1a", 16, 32, 16, 27, 0, 1},
    {"dec1b", 16, 0, 16, 27, 0, 1},   {"head", 16, 0, 4, 1, 0, 0},
};

int64_t layer_params(const LayerDef& d) {
    return (int64_t)d.cout * d.taps * (d.c1 + d.c2) + d.cout;
}

int64_t total_params() {
    int64_t p = 0;
    for (const LayerDef& d : kDefs) p += layer_params(d);
    return p;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

struct Layout {
    size_t theta, m, v, grad;
    size_t wp[kLayers], wt[kLayers];
    size_t act[kLayers];   // outputs (head: FP32 channel-first)
    size_t dact[kLayers];  // gradients of the pre-activations (none for the head)
    size_t in, pool[3], dpool[3], dcat[3];
    size_t partial, loss;
    size_t wpart;  // weight-gradient partial sums (the largest layer's, or the head's);
                   // also the 8-cell convolutions' partial sums (wpart_floats floats)
    int64_t wpart_floats;
    size_t total;
};

}  // namespace

struct lbm_nn {
    lbm_nn_config cfg;
    int lg0;
    char* ws;
    hipStream_t stream;
    Layout lay;
    int64_t P;
    int64_t off[kLayers];  // parameter offsets (weight, then bias)
    int t;                 // Adam steps taken
    int last_n;            // samples of the last forward pass

    template <typename T>
    T* at(size_t o) const { return (T*)(ws + o); }
    int lg(int layer) const { return lg0 - kDefs[layer].level; }
    ConvGeom geom(int layer, int n) const {
        const LayerDef& d = kDefs[layer];
        return make_geom(n, lg(layer), d.taps, d.c1, d.c2, d.cout);
    }
    int64_t cells(int layer, int n) const { return (int64_t)n << (3 * lg(layer)); }
};

namespace {

bool valid_config(const lbm_nn_config* c, std::string* why) {
    if (!c) return *why = "null configuration", false;
    if (c->grid < 8 || c->grid > 256 || (c->grid & (c->grid - 1)))
        return *why = "grid must be a power of two in [8, 256]", false;
    if (c->batch < 1 || c->batch > kMaxBatch) return *why = "batch must be in [1, 64]", false;
    if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) ||
        !(c->eps > 0))
        return *why = "Adam parameters out of range", false;
    return true;
}

Layout make_layout(const lbm_nn_config& c) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, kAlign);
        return at;
    };
    const int64_t P = total_params();
    L.theta = take(P * 4);
    L.m = take(P * 4);
    L.v = take(P * 4);
    L.grad = take(P * 4);
    const int lg0 = ilog2(c.grid), B = c.batch;
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef& d = kDefs[l];
        const ConvGeom g = make_geom(B, lg0 - d.level, d.taps, d.c1, d.c2, d.cout);
        L.wp[l] = take((size_t)g.coutp * g.kpad * 2);
        L.wt[l] = take((size_t)g.cinp * g.kpad_t * 2);
        const size_t cells = (size_t)B << (3 * (lg0 - d.level));
        const bool head = l == kLayers - 1;
        L.act[l] = head ? take(cells * 4 * 4) : take(cells * g.ys * 2);
        L.dact[l] = head ? 0 : take(cells * g.ys * 2);
    }
    const size_t c0 = (size_t)B << (3 * lg0);
    L.in = take(c0 * 8 * 2);
    const int pc[3] = {16, 32, 64};     // channels pooled after levels 0, 1, 2
    const int cc[3] = {48, 96, 192};    // concatenated inputs of dec1a, dec2a, dec3a
    for (int i = 0; i < 3; ++i) {
        const size_t coarse = (size_t)B << (3 * (lg0 - i - 1));
        L.pool[i] = take(coarse * pc[i] * 2);
        L.dpool[i] = take(coarse * pc[i] * 2);
        L.dcat[i] = take(((size_t)B << (3 * (lg0 - i))) * cc[i] * 2);
    }
    L.partial = take(((c0 + 255) / 256) * 8);
    L.loss = take(64);
    int64_t wpart = 0;
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef& d = kDefs[l];
        const ConvGeom g = make_geom(B, lg0 - d.level, d.taps, d.c1, d.c2, d.cout);
        wpart = std::max(wpart, l == kLayers - 1 ? head_scratch_floats(g)
                                                 : std::max(wgrad_scratch_floats(g),
                                                            conv_scratch_floats(g)));
    }
    L.wpart = take((size_t)wpart * 4);
    L.wpart_floats = wpart;
    L.total = o;
    return L;
}

lbm_status hipf(hipError_t e, const char* what) { return lbm::hip_fail(e, what); }

#define NN_TRY(expr, what)                         \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hipf(e_, what); \
    } while (0)

lbm_status pack_all(lbm_nn* nn) {
    ConvGeom g[kLayers];
    __bf16* wp[kLayers];
    __bf16* wt[kLayers];
    for (int l = 0; l < kLayers; ++l) {
        g[l] = nn->geom(l, 1);
        wp[l] = nn->at<__bf16>(nn->lay.wp[l]);
        wt[l] = nn->at<__bf16>(nn->lay.wt[l]);
    }
    NN_TRY(pack_weights(kLayers, g, nn->at<float>(nn->lay.theta), nn->off, wp, wt, nn->stream),
           "pack weights");
    return LBM_OK;
}

const float* bias_of(const lbm_nn* nn, int l) {
    const LayerDef& d = kDefs[l];
    return nn->at<float>(nn->lay.theta) + nn->off[l] + (int64_t)d.cout * d.taps * (d.c1 + d.c2);
}

// Inputs of layer l: (x1, x2) device pointers.
void layer_inputs(const lbm_nn* nn, int l, const __bf16** x1, const __bf16** x2) {
    const Layout& L = nn->lay;
    auto act = [&](int i) { return nn->at<__bf16>(L.act[i]); };
    *x2 = nullptr;
    switch (l) {
        case 0: *x1 = nn->at<__bf16>(L.in); break;
        case 2: *x1 = nn->at<__bf16>(L.pool[0]); break;
        case 4: *x1 = nn->at<__bf16>(L.pool[1]); break;
        case 6: *x1 = nn->at<__bf16>(L.pool[2]); break;
        case 9: *x1 = act(5), *x2 = act(8); break;
        case 11: *x1 = act(3), *x2 = act(10); break;
        case 13: *x1 = act(1), *x2 = act(12); break;
        default: *x1 = act(l - 1); break;
    }
}

// Forward pass up to the head's input act[head - 1].  The head runs where
// its output is used: into the caller's buffer (lbm_nn_forward), inside the
// loss and backward step, or into act[head] when that is asked for.
lbm_status forward(lbm_nn* nn, int n, const float* log10_ra) {
    const Layout& L = nn->lay;
    hipStream_t s = nn->stream;
    NN_TRY(make_inputs(n, nn->lg0, log10_ra, nn->at<__bf16>(L.in), s), "inputs");
    for (int l = 0; l < kLayers - 1; ++l) {
        const ConvGeom g = nn->geom(l, n);
        const __bf16 *x1, *x2;
        layer_inputs(nn, l, &x1, &x2);
        NN_TRY(conv_forward(g, x1, x2, nn->at<__bf16>(L.wp[l]), bias_of(nn, l), kDefs[l].relu,
                            nn->at<__bf16>(L.act[l]), nn->at<float>(L.wpart), L.wpart_floats, s),
               "conv forward");
        if (l == 1 || l == 3 || l == 5) {
            const int i = (l - 1) / 2;
            NN_TRY(pool_forward(n, nn->lg(l), kDefs[l].cout, nn->at<__bf16>(L.act[l]),
                                nn->at<__bf16>(L.pool[i]), s),
                   "pool");
        }
    }
    nn->last_n = n;
    return LBM_OK;
}

// Backward pass below the head, from the gradient in dact[head - 1] that
// the head's backward step wrote: gradients of the parameters of layers
// head - 1 .. 0 into grad.  Each dact[l] holds the gradient of layer l's
// pre-activation: the kernel that writes it applies the ReLU mask of act[l]
// once, so the convolutions read it unmasked.
lbm_status backward(lbm_nn* nn, int n) {
    const Layout& L = nn->lay;
    hipStream_t s = nn->stream;
    float* grad = nn->at<float>(L.grad);
    auto act = [&](int i) { return nn->at<__bf16>(L.act[i]); };
    auto dact = [&](int i) { return nn->at<__bf16>(L.dact[i]); };
    for (int l = kLayers - 2; l >= 0; --l) {
        const LayerDef& d = kDefs[l];
        const ConvGeom g = nn->geom(l, n);
        const __bf16 *x1, *x2;
        layer_inputs(nn, l, &x1, &x2);
        float* dw = grad + nn->off[l];
        float* db = dw + (int64_t)d.cout * d.taps * (d.c1 + d.c2);
        NN_TRY(conv_backward_weight(g, x1, x2, dact(l), nullptr, 0, dw, db,
                                    nn->at<float>(L.wpart), s),
               "weight grad");
        if (l == 0) break;
        // where the input gradient goes, and the ReLU mask it takes there
        __bf16* dx;
        const __bf16* dxmask = nullptr;
        switch (l) {
            case 2: dx = nn->at<__bf16>(L.dpool[0]); break;
            case 4: dx = nn->at<__bf16>(L.dpool[1]); break;
            case 6: dx = nn->at<__bf16>(L.dpool[2]); break;
            case 9: dx = nn->at<__bf16>(L.dcat[2]); break;
            case 11: dx = nn->at<__bf16>(L.dcat[1]); break;
            case 13: dx = nn->at<__bf16>(L.dcat[0]); break;
            default:
                dx = dact(l - 1);
                dxmask = kDefs[l - 1].relu ? act(l - 1) : nullptr;
                break;
        }
        // (the weight gradient above has finished with wpart: same stream)
        NN_TRY(conv_backward_data(g, dact(l), nn->at<__bf16>(L.wt[l]), dxmask, dx,
                                  nn->at<float>(L.wpart), L.wpart_floats, s),
               "data grad");
        if (l == 9 || l == 11 || l == 13) {
            // the upsampled half of the concatenation -> the coarse layer
            const int src = l == 9 ? 8 : l == 11 ? 10 : 12;
            NN_TRY(upsample_backward(n, nn->lg(l), d.c2, dx, g.cin, g.c1s,
                                     kDefs[src].relu ? act(src) : nullptr, dact(src), s),
                   "upsample backward");
        }
        if (l == 2 || l == 4 || l == 6) {
            // pooled input: the encoder layer before it also feeds a skip
            const int i = (l - 2) / 2;
            const int dec = l == 2 ? 13 : l == 4 ? 11 : 9;
            const ConvGeom gd = nn->geom(dec, n);
            NN_TRY(pool_backward_add(n, nn->lg(l - 1), kDefs[l - 1].cout,
                                     nn->at<__bf16>(L.dpool[i]), nn->at<__bf16>(L.dcat[i]),
                                     gd.cin, kDefs[l - 1].relu ? act(l - 1) : nullptr,
                                     dact(l - 1), s),
                   "pool backward");
        }
    }
    return LBM_OK;
}

lbm_status loss_and_backward(lbm_nn* nn, int n, const float* log10_ra, const float* targets,
                             const int32_t* idx, int64_t stride) {
    const Layout& L = nn->lay;
    lbm_status st = forward(nn, n, log10_ra);
    if (st != LBM_OK) return st;
    const int h = kLayers - 1;
    // (every entry of grad is written once below, by the head's sums and each
    // layer's weight-gradient reduction: no clearing)
    float* grad = nn->at<float>(L.grad);
    NN_TRY(head_backward(nn->geom(h, n), targets, idx, stride, nn->cfg.target_scale,
                         nn->at<__bf16>(L.act[h - 1]), nn->at<float>(L.theta) + nn->off[h],
                         bias_of(nn, h), nn->at<__bf16>(L.dact[h - 1]), grad + nn->off[h],
                         nn->at<float>(L.wpart), nn->at<double>(L.partial),
                         nn->at<double>(L.loss), nn->stream),
           "loss and head backward");
    return backward(nn, n);
}

lbm_status read_loss(lbm_nn* nn, int n, double* loss) {
    double sum = 0;
    NN_TRY(hipMemcpyAsync(&sum, nn->at<double>(nn->lay.loss), sizeof sum, hipMemcpyDeviceToHost,
                          nn->stream),
           "loss copy");
    NN_TRY(hipStreamSynchronize(nn->stream), "loss sync");
    *loss = sum / ((double)n * 4.0 * (double)((int64_t)1 << (3 * nn->lg0)));
    return LBM_OK;
}

lbm_status check_call(lbm_nn* nn, int n, const float* lra) {
    if (!nn) return lbm::fail(LBM_ERR_ARG, "null network");
    if (n < 1 || n > nn->cfg.batch) return lbm::fail(LBM_ERR_ARG, "n must be in [1, batch]");
    if (!lra) return lbm::fail(LBM_ERR_ARG, "null log10_ra");
    return LBM_OK;
}

lbm_status check_targets(const float* targets, int64_t count, const int32_t* idx, int n,
                         int64_t stride, int64_t need) {
    if (!targets || !idx) return lbm::fail(LBM_ERR_ARG, "null targets");
    if (stride < need) return lbm::fail(LBM_ERR_ARG, "target_stride below 4 G^3");
    if (count < 1) return lbm::fail(LBM_ERR_ARG, "target_count must be positive");
    for (int i = 0; i < n; ++i)
        if (idx[i] < 0 || idx[i] >= count)
            return lbm::fail(LBM_ERR_ARG, "target index outside [0, target_count)");
    return LBM_OK;
}

}  // namespace

extern "C" {

int64_t lbm_nn_param_count(void) { return total_params(); }

size_t lbm_nn_workspace_bytes(const lbm_nn_config* c) {
    std::string why;
    if (!valid_config(c, &why)) {
        lbm::fail(LBM_ERR_ARG, why);
        return 0;
    }
    return make_layout(*c).total;
}

lbm_status lbm_nn_create(const lbm_nn_config* c, void* workspace, size_t bytes, void* stream,
                         lbm_nn** out) {
    std::string why;
    if (!out) return lbm::fail(LBM_ERR_ARG, "null output");
    *out = nullptr;
    if (!valid_config(c, &why)) return lbm::fail(LBM_ERR_ARG, why);
    const Layout L = make_layout(*c);
    if (!workspace || bytes < L.total || ((uintptr_t)workspace % kAlign))
        return lbm::fail(LBM_ERR_ARG, "workspace missing, too small or not 256-byte aligned");
    lbm_nn* nn = new (std::nothrow) lbm_nn;
    if (!nn) return lbm::fail(LBM_ERR_ARG, "out of host memory");
    nn->cfg = *c;
    nn->lg0 = ilog2(c->grid);
    nn->ws = (char*)workspace;
    nn->stream = (hipStream_t)stream;
    nn->lay = L;
    nn->P = total_params();
    int64_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        nn->off[l] = o;
        o += layer_params(kDefs[l]);
    }
    nn->t = 0;
    nn->last_n = 0;
    // parameters, moments and packed weights start at zero
    hipError_t e = fill_zero_f32(nn->at<float>(L.theta), nn->P, nn->stream);
    if (e == hipSuccess) e = fill_zero_f32(nn->at<float>(L.m), nn->P, nn->stream);
    if (e == hipSuccess) e = fill_zero_f32(nn->at<float>(L.v), nn->P, nn->stream);
    if (e != hipSuccess) {
        delete nn;
        return hipf(e, "nn init");
    }
    lbm_status st = pack_all(nn);
    if (st != LBM_OK) {
        delete nn;
        return st;
    }
    *out = nn;
    return LBM_OK;
}

lbm_status lbm_nn_destroy(lbm_nn* nn) {
    delete nn;
    return LBM_OK;
}

lbm_status lbm_nn_set_params(lbm_nn* nn, const float* params) {
    if (!nn || !params) return lbm::fail(LBM_ERR_ARG, "null argument");
    NN_TRY(hipMemcpyAsync(nn->at<float>(nn->lay.theta), params, nn->P * 4,
                          hipMemcpyDeviceToDevice, nn->stream),
           "set params");
    NN_TRY(fill_zero_f32(nn->at<float>(nn->lay.m), nn->P, nn->stream), "reset m");
    NN_TRY(fill_zero_f32(nn->at<float>(nn->lay.v), nn->P, nn->stream), "reset v");
    nn->t = 0;
    return pack_all(nn);
}

lbm_status lbm_nn_get_params(lbm_nn* nn, float* params) {
    if (!nn || !params) return lbm::fail(LBM_ERR_ARG, "null argument");
    NN_TRY(hipMemcpyAsync(params, nn->at<float>(nn->lay.theta), nn->P * 4,
                          hipMemcpyDeviceToDevice, nn->stream),
           "get params");
    return LBM_OK;
}

lbm_status lbm_nn_forward(lbm_nn* nn, int32_t n, const float* log10_ra, float* out,
                          const float* out_scale) {
    lbm_status st = check_call(nn, n, log10_ra);
    if (st != LBM_OK) return st;
    if (!out) return lbm::fail(LBM_ERR_ARG, "null output");
    st = forward(nn, n, log10_ra);
    if (st != LBM_OK) return st;
    // the head, into the caller's buffer with the scale
    const int h = kLayers - 1;
    NN_TRY(head_forward(nn->geom(h, n), nn->at<__bf16>(nn->lay.act[h - 1]),
                        nn->at<float>(nn->lay.theta) + nn->off[h], bias_of(nn, h), out_scale, out,
                        nn->stream),
           "head");
    return LBM_OK;
}

lbm_status lbm_nn_gradient(lbm_nn* nn, int32_t n, const float* log10_ra, const float* targets,
                           int64_t target_count, const int32_t* target_index,
                           int64_t target_stride, float* grad, double* loss) {
    lbm_status st = check_call(nn, n, log10_ra);
    if (st != LBM_OK) return st;
    st = check_targets(targets, target_count, target_index, n, target_stride,
                       (int64_t)4 << (3 * nn->lg0));
    if (st != LBM_OK) return st;
    if (!loss) return lbm::fail(LBM_ERR_ARG, "null loss");
    st = loss_and_backward(nn, n, log10_ra, targets, target_index, target_stride);
    if (st != LBM_OK) return st;
    if (grad)
        NN_TRY(hipMemcpyAsync(grad, nn->at<float>(nn->lay.grad), nn->P * 4,
                              hipMemcpyDeviceToDevice, nn->stream),
               "grad copy");
    return read_loss(nn, n, loss);
}

lbm_status lbm_nn_train_step(lbm_nn* nn, int32_t n, const float* log10_ra,
                             const float* targets, int64_t target_count,
                             const int32_t* target_index, int64_t target_stride, double* loss) {
    lbm_status st = check_call(nn, n, log10_ra);
    if (st != LBM_OK) return st;
    st = check_targets(targets, target_count, target_index, n, target_stride,
                       (int64_t)4 << (3 * nn->lg0));
    if (st != LBM_OK) return st;
    st = loss_and_backward(nn, n, log10_ra, targets, target_index, target_stride);
    if (st != LBM_OK) return st;
    nn->t += 1;
    NN_TRY(adam_update(nn->P, nn->at<float>(nn->lay.theta), nn->at<float>(nn->lay.m),
                       nn->at<float>(nn->lay.v), nn->at<float>(nn->lay.grad), nn->t, nn->cfg.lr,
                       nn->cfg.beta1, nn->cfg.beta2, nn->cfg.eps, nn->stream),
           "adam");
    st = pack_all(nn);
    if (st != LBM_OK) return st;
    return loss ? read_loss(nn, n, loss) : LBM_OK;
}

lbm_status lbm_nn_set_lr(lbm_nn* nn, float lr) {
    if (!nn || !(lr > 0)) return lbm::fail(LBM_ERR_ARG, "lr must be positive");
    nn->cfg.lr = lr;
    return LBM_OK;
}

lbm_status lbm_nn_activation(lbm_nn* nn, int32_t layer, int32_t n, float* out) {
    if (!nn || !out) return lbm::fail(LBM_ERR_ARG, "null argument");
    if (layer < 0 || layer >= kLayers) return lbm::fail(LBM_ERR_ARG, "layer out of range");
    if (nn->last_n < 1) return lbm::fail(LBM_ERR_STATE, "no forward pass yet");
    if (n != nn->last_n) return lbm::fail(LBM_ERR_ARG, "n differs from the last forward pass");
    if (layer == kLayers - 1) {
        // the head's unscaled output, from its input of the last forward pass
        NN_TRY(head_forward(nn->geom(layer, n), nn->at<__bf16>(nn->lay.act[layer - 1]),
                            nn->at<float>(nn->lay.theta) + nn->off[layer], bias_of(nn, layer),
                            nullptr, nn->at<float>(nn->lay.act[layer]), nn->stream),
               "head forward");
        NN_TRY(cf_to_cl(nn->at<float>(nn->lay.act[layer]), n, nn->cells(layer, 1), 4, out,
                        nn->stream),
               "activation");
        return LBM_OK;
    }
    const ConvGeom g = nn->geom(layer, n);
    NN_TRY(bf16_to_f32(nn->at<__bf16>(nn->lay.act[layer]), nn->cells(layer, n), g.ys, g.cout, out,
                       nn->stream),
           "activation");
    return LBM_OK;
}

lbm_status lbm_nn_flops(const lbm_nn* nn, int32_t n, double* fwd, double* train) {
    if (!nn || !fwd || !train) return lbm::fail(LBM_ERR_ARG, "null argument");
    double f = 0, b = 0;
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef& d = kDefs[l];
        const double macs =
            (double)nn->cells(l, n) * d.cout * d.taps * (double)(d.c1 + d.c2);
        f += 2 * macs;
        b += 2 * macs * (l == 0 ? 1 : 2);  // weight gradient (+ input gradient)
    }
    *fwd = f;
    *train = f + b;
    return LBM_OK;
}

}  // extern "C"
