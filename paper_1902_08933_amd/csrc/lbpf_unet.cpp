// Learned surrogate: a 4-level convolutional U-Net that maps the fields (phi, u_x, u_y, p) of
// the solver at time t to time t + K (K time steps of the LB solver), trained on trajectories
// the solver generates. BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
// weights and Adam moments. Host side of the C ABI declared in include/lbpf.h.
//
// Architecture (c_l = base_ch << l, circular padding, 3x3 convolutions unless noted):
//   E0 = relu(conv(X, 16 -> c0))            X: input zero-padded to 16 channels, level 0
//   E1 = relu(conv(pool(E0), c0 -> c1))     level 1 (pool: 2x2 average)
//   E2 = relu(conv(pool(E1), c1 -> c2))     level 2
//   E3 = relu(conv(pool(E2), c2 -> c3))     level 3 (bottleneck)
//   D2 = relu(conv([up(E3), E2], c3+c2 -> c2))   (up: nearest 2x; [a, b]: channel concat)
//   D1 = relu(conv([up(D2), E1], c2+c1 -> c1))
//   D0 = relu(conv([up(D1), E0], c1+c0 -> c0))
//   Y  = conv1x1(D0, c0 -> 16); prediction = input + Y[:, :in_ch]
// The encoder outputs are written straight into the second half of the concat buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "lbpf.h"

#include "lbpf_unet_ops.hpp"

using namespace lbpf;

namespace {

constexpr int kLayers = 8;         // e0 e1 e2 e3 d2 d1 d0 head
constexpr int kLossBlocks = 1024;  // partial sums of the loss

struct Layer {
    int cin, cout, ks;
    long long woff, boff;  // offsets of weights and bias in the flat parameter vector
};

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

struct Geometry {
    int c[4];
    Layer layer[kLayers];
    long long nparam;
    long long npix0;  // max_batch * max_h * max_w
    long long max_layer_w;
};

Geometry make_geometry(const lbpf_unet_cfg* cfg) {
    Geometry g{};
    for (int l = 0; l < 4; ++l) g.c[l] = cfg->base_ch << l;
    const int ci[kLayers] = {16, g.c[0], g.c[1], g.c[2], g.c[3] + g.c[2], g.c[2] + g.c[1], g.c[1] + g.c[0], g.c[0]};
    const int co[kLayers] = {g.c[0], g.c[1], g.c[2], g.c[3], g.c[2], g.c[1], g.c[0], 16};
    long long off = 0;
    g.max_layer_w = 0;
    for (int i = 0; i < kLayers; ++i) {
        Layer& L = g.layer[i];
        L.cin = ci[i];
        L.cout = co[i];
        L.ks = (i == kLayers - 1) ? 1 : 3;
        L.woff = off;
        off += (long long)L.cout * L.ks * L.ks * L.cin;
        L.boff = off;
        off += L.cout;
        const long long nw = (long long)L.cout * L.ks * L.ks * L.cin;
        if (nw > g.max_layer_w) g.max_layer_w = nw;
    }
    g.nparam = off;
    g.npix0 = (long long)cfg->max_batch * cfg->max_h * cfg->max_w;
    return g;
}

// activation buffers (bf16, channels per pixel at their level)
enum Buf { X0, U0, P1, U1, P2, U2, P3, E3, D2, D1, D0, YH, kNumBufs };

struct BufSpec { int level; int ch; };

void buf_specs(const Geometry& g, BufSpec* s) {
    s[X0] = {0, 16};
    s[U0] = {0, g.c[1] + g.c[0]};
    s[P1] = {1, g.c[0]};
    s[U1] = {1, g.c[2] + g.c[1]};
    s[P2] = {2, g.c[1]};
    s[U2] = {2, g.c[3] + g.c[2]};
    s[P3] = {3, g.c[2]};
    s[E3] = {3, g.c[3]};
    s[D2] = {2, g.c[2]};
    s[D1] = {1, g.c[1]};
    s[D0] = {0, g.c[0]};
    s[YH] = {0, 16};
}

}  // namespace

struct lbpf_unet {
    lbpf_unet_cfg cfg;
    Geometry g;
    BufSpec spec[kNumBufs];
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    // parameters
    float* w32;    // master weights
    bf16* wbf;     // bf16 copy
    bf16* wflip;   // flipped weights for dgrad
    float* grad;
    float* adam_m;
    float* adam_v;
    int64_t adam_t;
    // activations and gradients
    bf16* act[kNumBufs];
    bf16* gact[kNumBufs];
    float* head32;   // FP32 head output [npix0][16]
    double* loss_part;
    float* wpart;    // wgrad partials
    float* bpart;
    float* wch;      // loss channel weights (16 floats, device)
    float wch_host[16];
    std::string err;
};

static thread_local std::string g_unet_err;

static lbpf_status ufail(lbpf_unet* u, lbpf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (u) u->err = buf;
    else g_unet_err = buf;
    return s;
}

static const char* validate_cfg(const lbpf_unet_cfg* c) {
    if (!c) return "cfg is NULL";
    if (c->in_ch < 1 || c->in_ch > 16) return "in_ch must be in 1..16";
    if (c->base_ch < 16 || c->base_ch % 16 != 0 || c->base_ch > 128) return "base_ch must be 16, 32, ..., 128";
    if (c->max_batch < 1 || c->max_h < 8 || c->max_w < 8) return "max_batch >= 1 and max_h, max_w >= 8 required";
    if (c->max_h % 8 != 0 || c->max_w % 8 != 0) return "max_h and max_w must be multiples of 8";
    if (c->wgrad_chunks < 0 || c->wgrad_chunks > 1024) return "wgrad_chunks must be in 0..1024";
    return nullptr;
}

static size_t layout(const lbpf_unet_cfg* cfg, lbpf_unet* u) {
    Geometry g = make_geometry(cfg);
    BufSpec spec[kNumBufs];
    buf_specs(g, spec);
    const bool train = cfg->train != 0;
    const int chunks = cfg->wgrad_chunks > 0 ? cfg->wgrad_chunks : 64;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += a256(bytes); return o; };
    const size_t o_w32 = take(g.nparam * 4), o_wbf = take(g.nparam * 2);
    const size_t o_flip = train ? take(g.nparam * 2) : 0;
    const size_t o_grad = train ? take(g.nparam * 4) : 0;
    const size_t o_m = train ? take(g.nparam * 4) : 0, o_v = train ? take(g.nparam * 4) : 0;
    size_t o_act[kNumBufs], o_gact[kNumBufs];
    for (int b = 0; b < kNumBufs; ++b) {
        const long long pix = g.npix0 >> (2 * spec[b].level);
        o_act[b] = take((size_t)pix * spec[b].ch * 2);
        o_gact[b] = train ? take((size_t)pix * spec[b].ch * 2) : 0;
    }
    const size_t o_head = take((size_t)g.npix0 * 16 * 4);
    const size_t o_loss = take(kLossBlocks * 8);
    const size_t o_wpart = train ? take((size_t)chunks * g.max_layer_w * 4) : 0;
    const size_t o_bpart = train ? take((size_t)chunks * (cfg->base_ch << 3) * 4) : 0;
    const size_t o_wch = take(16 * 4);
    if (u) {
        u->g = g;
        for (int b = 0; b < kNumBufs; ++b) u->spec[b] = spec[b];
        u->w32 = (float*)(u->ws + o_w32);
        u->wbf = (bf16*)(u->ws + o_wbf);
        u->wflip = train ? (bf16*)(u->ws + o_flip) : nullptr;
        u->grad = train ? (float*)(u->ws + o_grad) : nullptr;
        u->adam_m = train ? (float*)(u->ws + o_m) : nullptr;
        u->adam_v = train ? (float*)(u->ws + o_v) : nullptr;
        for (int b = 0; b < kNumBufs; ++b) {
            u->act[b] = (bf16*)(u->ws + o_act[b]);
            u->gact[b] = train ? (bf16*)(u->ws + o_gact[b]) : nullptr;
        }
        u->head32 = (float*)(u->ws + o_head);
        u->loss_part = (double*)(u->ws + o_loss);
        u->wpart = train ? (float*)(u->ws + o_wpart) : nullptr;
        u->bpart = train ? (float*)(u->ws + o_bpart) : nullptr;
        u->wch = (float*)(u->ws + o_wch);
    }
    return off;
}

#define UCHK(expr)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return ufail(u, LBPF_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static lbpf_status check_dims(lbpf_unet* u, int n, int h, int w) {
    if (n < 1 || h < 8 || w < 8 || h % 8 || w % 8)
        return ufail(u, LBPF_E_INVALID, "n >= 1 and h, w multiples of 8 required (got %d, %d, %d)", n, h, w);
    if ((long long)n * h * w > u->g.npix0)
        return ufail(u, LBPF_E_NOMEM, "n*h*w = %lld exceeds the workspace (%lld pixels)", (long long)n * h * w, u->g.npix0);
    return LBPF_OK;
}

// Largest number of pixel chunks whose weight-gradient partials of layer L fit the partial
// buffers (sized for wgrad_chunks chunks of the largest layer).
static int wgrad_max_chunks(const lbpf_unet* u, const Layer& L) {
    const long long cfg_chunks = u->cfg.wgrad_chunks > 0 ? u->cfg.wgrad_chunks : 64;
    const long long by_w = cfg_chunks * u->g.max_layer_w / ((long long)L.cout * L.ks * L.ks * L.cin);
    const long long by_b = cfg_chunks * (u->cfg.base_ch << 3) / L.cout;
    const long long m = by_w < by_b ? by_w : by_b;
    return (int)(m > (1 << 20) ? (1 << 20) : m);
}

// Forward pass. The decoder convolutions read the upsampled half of their input straight from
// the lower level (the concat is never formed). With `pred` (inference) the 1x1 head writes the
// prediction input + Y[:, :in_ch] and nothing else; without it (loss and gradients) the head's
// outputs are kept for the loss, and the upsampled halves of the concat buffers are written
// out as well, since the weight gradients read them.
static lbpf_status forward(lbpf_unet* u, const float* in, int n, int h, int w, float* pred) {
    const Geometry& g = u->g;
    hipStream_t st = u->stream;
    const long long np0 = (long long)n * h * w;
    const int* c = g.c;
    const int su0 = c[1] + c[0], su1 = c[2] + c[1], su2 = c[3] + c[2];
    const Layer* L = g.layer;
    const bool keep = pred == nullptr;
    auto W = [&](int i) { return u->wbf + L[i].woff; };
    auto B = [&](int i) { return u->w32 + L[i].boff; };
    // the first layer reads the FP32 input itself; the packed bf16 copy is needed only by the
    // weight gradient of that layer (and for inputs of more than 4 fields)
    const bool direct_in = !keep && u->cfg.in_ch <= 4;
    if (!direct_in) UCHK(unet_pack_input(in, u->cfg.in_ch, u->act[X0], np0, st));
    // encoder: E_l goes into the second part of the concat buffer of its level, and its 2x2
    // average pool P_{l+1} (the next layer's input) is written by the same kernel. In inference
    // the concat is never formed, so E_l is stored dense at the start of that buffer instead
    // (its own channel stride): the decoder's reads of it, and the encoder's writes, are then
    // whole cache lines.
    const bool dense = !keep;
    auto enc = [&](int i, Buf xin, int cin, int sx, Buf out, int so, int oo, Buf pool, int cout,
                   int lev) -> lbpf_status {
        ConvArgs a{};
        a.x = u->act[xin]; a.xs = sx; a.xo = 0;
        a.Cin = cin; a.w = W(i); a.bias = B(i);
        if (i == 0 && direct_in) { a.x = nullptr; a.xin = in; a.xin_c = u->cfg.in_ch; }
        a.y = u->act[out]; a.ys = so; a.yo = oo;
        if (pool != kNumBufs) { a.yp = u->act[pool]; a.yps = cout; a.ypo = 0; }
        a.Cout = cout; a.N = n; a.H = h >> lev; a.W = w >> lev;
        UCHK(unet_conv(3, true, a, st));
        return LBPF_OK;
    };
    lbpf_status s;
    if ((s = enc(0, X0, 16, 16, U0, dense ? c[0] : su0, dense ? 0 : c[1], P1, c[0], 0))) return s;
    if ((s = enc(1, P1, c[0], c[0], U1, dense ? c[1] : su1, dense ? 0 : c[2], P2, c[1], 1))) return s;
    if ((s = enc(2, P2, c[1], c[1], U2, dense ? c[2] : su2, dense ? 0 : c[3], P3, c[2], 2))) return s;
    if ((s = enc(3, P3, c[2], c[2], E3, c[3], 0, kNumBufs, c[3], 3))) return s;
    // decoder: layer i reads [up(low), skip] with low = (buffer, channels), skip at offset cl of
    // the concat buffer cat (stride scat), at level lev
    auto dec = [&](int i, Buf low, int cl, Buf cat, int scat, Buf out, int cout, int lev) -> lbpf_status {
        if (keep) UCHK(unet_upsample(u->act[low], cl, 0, u->act[cat], scat, 0, cl, n, h >> lev, w >> lev, st));
        ConvArgs a{};
        a.x = u->act[cat]; a.xs = dense ? scat - cl : scat; a.xo = dense ? 0 : cl;
        a.xl = u->act[low]; a.xls = cl; a.xlo = 0; a.Cl = cl;
        a.Cin = scat; a.w = W(i); a.bias = B(i);
        a.y = u->act[out]; a.ys = cout; a.yo = 0;
        a.Cout = cout; a.N = n; a.H = h >> lev; a.W = w >> lev;
        UCHK(unet_conv(3, true, a, st));
        return LBPF_OK;
    };
    if ((s = dec(4, E3, c[3], U2, su2, D2, c[2], 2))) return s;
    if ((s = dec(5, D2, c[2], U1, su1, D1, c[1], 1))) return s;
    if (!keep && c[0] <= 32) {
        // inference: D0 stays on chip; its workgroups apply the 1x1 head and write the prediction
        ConvArgs a{};
        a.x = u->act[U0]; a.xs = c[0]; a.xo = 0;  // dense (inference)
        a.xl = u->act[D1]; a.xls = c[1]; a.xlo = 0; a.Cl = c[1];
        a.Cin = su0; a.w = W(6); a.bias = B(6);
        a.hw = W(7); a.hb = B(7); a.res = in; a.pred = pred; a.rc = u->cfg.in_ch;
        a.Cout = c[0]; a.N = n; a.H = h; a.W = w;
        UCHK(unet_conv(3, true, a, st));
        return LBPF_OK;
    }
    if ((s = dec(6, D1, c[1], U0, su0, D0, c[0], 0))) return s;
    ConvArgs a{};
    a.x = u->act[D0]; a.xs = c[0]; a.xo = 0;
    a.Cin = c[0]; a.w = W(7); a.bias = B(7);
    a.Cout = 16; a.N = n; a.H = h; a.W = w;
    if (keep) {
        a.y = u->act[YH]; a.ys = 16; a.yo = 0;
        a.yf = u->head32;
    } else {
        a.res = in; a.pred = pred; a.rc = u->cfg.in_ch;
    }
    UCHK(unet_conv(1, false, a, st));
    return LBPF_OK;
}

static lbpf_status loss_reduce(lbpf_unet* u, long long npix, double* loss_host) {
    std::vector<double> part(kLossBlocks);
    UCHK(hipMemcpyAsync(part.data(), u->loss_part, kLossBlocks * 8, hipMemcpyDeviceToHost, u->stream));
    UCHK(hipStreamSynchronize(u->stream));
    double s = 0.0;
    for (double v : part) s += v;  // fixed order
    if (loss_host) *loss_host = s / ((double)npix * u->cfg.in_ch);
    return LBPF_OK;
}

// gradient of one convolution layer i whose input is buffer (xb, xs, xo, cin) at level lev,
// output gradient in gact[yb] (channel stride ys, offset 0); writes dW, db into grad and, when
// dxb >= 0, the data gradient into gact[dxb] (stride dxs)
static lbpf_status conv_backward(lbpf_unet* u, int i, int lev, int n, int h, int w, Buf yb, int ys,
                                 Buf xb, int xs, int xo, int dxb, int dxs) {
    const Layer& L = u->g.layer[i];
    hipStream_t st = u->stream;
    const int H = h >> lev, Wd = w >> lev;
    UCHK(unet_conv_wgrad(L.ks, u->gact[yb], ys, 0, L.cout, u->act[xb], xs, xo, L.cin, n, H, Wd, wgrad_max_chunks(u, L),
                         u->wpart, u->bpart, u->grad + L.woff, u->grad + L.boff, st));
    if (dxb >= 0) {
        UCHK(unet_flip_weights(u->wbf + L.woff, u->wflip + L.woff, L.cout, L.cin, L.ks * L.ks, st));
        UCHK(unet_conv_fwd(L.ks, false, u->gact[yb], ys, 0, L.cout, u->wflip + L.woff, nullptr,
                           u->gact[dxb], dxs, 0, L.cin, nullptr, n, H, Wd, st));
    }
    return LBPF_OK;
}

static lbpf_status backward(lbpf_unet* u, int n, int h, int w) {
    const int* c = u->g.c;
    const int su0 = c[1] + c[0], su1 = c[2] + c[1], su2 = c[3] + c[2];
    hipStream_t st = u->stream;
    const long long np0 = (long long)n * h * w, np1 = np0 / 4, np2 = np0 / 16, np3 = np0 / 64;
    lbpf_status s;
    // head (1x1) -> dD0
    if ((s = conv_backward(u, 7, 0, n, h, w, YH, 16, D0, c[0], 0, D0, c[0]))) return s;
    UCHK(unet_relu_bwd(u->gact[D0], c[0], 0, u->act[D0], c[0], 0, c[0], np0, st));
    // d0: input U0 -> dU0
    if ((s = conv_backward(u, 6, 0, n, h, w, D0, c[0], U0, su0, 0, U0, su0))) return s;
    UCHK(unet_upsample_bwd(u->gact[U0], su0, 0, u->gact[D1], c[1], 0, c[1], n, h, w, st));
    UCHK(unet_relu_bwd(u->gact[D1], c[1], 0, u->act[D1], c[1], 0, c[1], np1, st));
    // d1: input U1
    if ((s = conv_backward(u, 5, 1, n, h, w, D1, c[1], U1, su1, 0, U1, su1))) return s;
    UCHK(unet_upsample_bwd(u->gact[U1], su1, 0, u->gact[D2], c[2], 0, c[2], n, h / 2, w / 2, st));
    UCHK(unet_relu_bwd(u->gact[D2], c[2], 0, u->act[D2], c[2], 0, c[2], np2, st));
    // d2: input U2
    if ((s = conv_backward(u, 4, 2, n, h, w, D2, c[2], U2, su2, 0, U2, su2))) return s;
    UCHK(unet_upsample_bwd(u->gact[U2], su2, 0, u->gact[E3], c[3], 0, c[3], n, h / 4, w / 4, st));
    UCHK(unet_relu_bwd(u->gact[E3], c[3], 0, u->act[E3], c[3], 0, c[3], np3, st));
    // e3: input P3 -> dP3, then into the E2 part of dU2
    if ((s = conv_backward(u, 3, 3, n, h, w, E3, c[3], P3, c[2], 0, P3, c[2]))) return s;
    UCHK(unet_avgpool_bwd_add(u->gact[P3], c[2], 0, u->gact[U2], su2, c[3], c[2], n, h / 4, w / 4, st));
    // the E2 gradient lives at offset c3 of dU2; relu, then e2's backward needs it at offset 0
    UCHK(unet_relu_bwd(u->gact[U2], su2, c[3], u->act[U2], su2, c[3], c[2], np2, st));
    {
        const Layer& L = u->g.layer[2];
        const int chunks = wgrad_max_chunks(u, L);
        UCHK(unet_conv_wgrad(3, u->gact[U2], su2, c[3], L.cout, u->act[P2], c[1], 0, L.cin, n, h / 4, w / 4,
                             chunks, u->wpart, u->bpart, u->grad + L.woff, u->grad + L.boff, st));
        UCHK(unet_flip_weights(u->wbf + L.woff, u->wflip + L.woff, L.cout, L.cin, 9, st));
        UCHK(unet_conv_fwd(3, false, u->gact[U2] + c[3], su2, 0, L.cout, u->wflip + L.woff, nullptr,
                           u->gact[P2], c[1], 0, L.cin, nullptr, n, h / 4, w / 4, st));
    }
    UCHK(unet_avgpool_bwd_add(u->gact[P2], c[1], 0, u->gact[U1], su1, c[2], c[1], n, h / 2, w / 2, st));
    UCHK(unet_relu_bwd(u->gact[U1], su1, c[2], u->act[U1], su1, c[2], c[1], np1, st));
    {
        const Layer& L = u->g.layer[1];
        const int chunks = wgrad_max_chunks(u, L);
        UCHK(unet_conv_wgrad(3, u->gact[U1], su1, c[2], L.cout, u->act[P1], c[0], 0, L.cin, n, h / 2, w / 2,
                             chunks, u->wpart, u->bpart, u->grad + L.woff, u->grad + L.boff, st));
        UCHK(unet_flip_weights(u->wbf + L.woff, u->wflip + L.woff, L.cout, L.cin, 9, st));
        UCHK(unet_conv_fwd(3, false, u->gact[U1] + c[2], su1, 0, L.cout, u->wflip + L.woff, nullptr,
                           u->gact[P1], c[0], 0, L.cin, nullptr, n, h / 2, w / 2, st));
    }
    UCHK(unet_avgpool_bwd_add(u->gact[P1], c[0], 0, u->gact[U0], su0, c[1], c[0], n, h, w, st));
    UCHK(unet_relu_bwd(u->gact[U0], su0, c[1], u->act[U0], su0, c[1], c[0], np0, st));
    {
        const Layer& L = u->g.layer[0];
        const int chunks = wgrad_max_chunks(u, L);
        UCHK(unet_conv_wgrad(3, u->gact[U0], su0, c[1], L.cout, u->act[X0], 16, 0, L.cin, n, h, w,
                             chunks, u->wpart, u->bpart, u->grad + L.woff, u->grad + L.boff, st));
    }
    return LBPF_OK;
}

extern "C" {

lbpf_status lbpf_unet_workspace_size(const lbpf_unet_cfg* cfg, size_t* bytes) {
    if (const char* why = validate_cfg(cfg)) return ufail(nullptr, LBPF_E_INVALID, "%s", why);
    if (!bytes) return ufail(nullptr, LBPF_E_INVALID, "bytes is NULL");
    *bytes = layout(cfg, nullptr);
    return LBPF_OK;
}

lbpf_status lbpf_unet_create(const lbpf_unet_cfg* cfg, void* workspace, size_t workspace_bytes,
                             void* hip_stream, lbpf_unet** out) {
    if (!out) return ufail(nullptr, LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* why = validate_cfg(cfg)) return ufail(nullptr, LBPF_E_INVALID, "%s", why);
    const size_t need = layout(cfg, nullptr);
    if (!workspace || ((uintptr_t)workspace) % 256) return ufail(nullptr, LBPF_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return ufail(nullptr, LBPF_E_NOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    lbpf_unet* u = new (std::nothrow) lbpf_unet();
    if (!u) return ufail(nullptr, LBPF_E_NOMEM, "host allocation failed");
    u->cfg = *cfg;
    u->ws = (char*)workspace;
    u->ws_bytes = workspace_bytes;
    u->stream = (hipStream_t)hip_stream;
    layout(cfg, u);
    u->adam_t = 0;
    // He-normal initial weights from a seeded generator, zero biases, zero head (the initial
    // network predicts no change)
    std::vector<float> w(u->g.nparam, 0.0f);
    std::mt19937_64 rng(cfg->seed);
    for (int i = 0; i < kLayers - 1; ++i) {
        const Layer& L = u->g.layer[i];
        const int fan_in = L.ks * L.ks * (i == 0 ? cfg->in_ch : L.cin);
        std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / (float)fan_in));
        const long long nw = (long long)L.cout * L.ks * L.ks * L.cin;
        for (long long k = 0; k < nw; ++k) {
            const int ci = (int)(k % L.cin);
            w[L.woff + k] = (i == 0 && ci >= cfg->in_ch) ? 0.0f : nd(rng);
        }
    }
    for (int c = 0; c < 16; ++c) u->wch_host[c] = c < cfg->in_ch ? 1.0f : 0.0f;
    lbpf_status s = lbpf_unet_set_params(u, nullptr);
    hipError_t e = hipMemcpy(u->w32, w.data(), u->g.nparam * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(u->wch, u->wch_host, 64, hipMemcpyHostToDevice);
    if (s == LBPF_OK && e == hipSuccess) s = lbpf_unet_set_params(u, u->w32);
    if (s != LBPF_OK || e != hipSuccess) {
        g_unet_err = u->err.empty() ? hipGetErrorString(e) : u->err;
        delete u;
        return s != LBPF_OK ? s : LBPF_E_HIP;
    }
    *out = u;
    return LBPF_OK;
}

int64_t lbpf_unet_param_count(const lbpf_unet* u) { return u ? u->g.nparam : -1; }

lbpf_status lbpf_unet_layer(const lbpf_unet* u, int32_t i, int64_t* woff, int64_t* boff,
                            int32_t* cout, int32_t* ks, int32_t* cin) {
    if (!u || i < 0 || i >= kLayers) return LBPF_E_INVALID;
    const Layer& L = u->g.layer[i];
    if (woff) *woff = L.woff;
    if (boff) *boff = L.boff;
    if (cout) *cout = L.cout;
    if (ks) *ks = L.ks;
    if (cin) *cin = L.cin;
    return LBPF_OK;
}

lbpf_status lbpf_unet_set_params(lbpf_unet* u, const float* src) {
    if (!u) return LBPF_E_INVALID;
    u->err.clear();
    if (!src) return LBPF_OK;
    const long long n = u->g.nparam;
    if (src != u->w32) UCHK(hipMemcpyAsync(u->w32, src, n * 4, hipMemcpyDeviceToDevice, u->stream));
    UCHK(unet_to_bf16(u->w32, u->wbf, n, u->stream));
    if (u->adam_m) {
        UCHK(hipMemsetAsync(u->adam_m, 0, n * 4, u->stream));
        UCHK(hipMemsetAsync(u->adam_v, 0, n * 4, u->stream));
    }
    u->adam_t = 0;
    UCHK(hipStreamSynchronize(u->stream));
    return LBPF_OK;
}

lbpf_status lbpf_unet_get_params(lbpf_unet* u, float* dst) {
    if (!u || !dst) return LBPF_E_INVALID;
    u->err.clear();
    UCHK(hipMemcpyAsync(dst, u->w32, u->g.nparam * 4, hipMemcpyDeviceToDevice, u->stream));
    return LBPF_OK;
}

lbpf_status lbpf_unet_set_loss_weights(lbpf_unet* u, const float* host_w) {
    if (!u || !host_w) return LBPF_E_INVALID;
    u->err.clear();
    for (int c = 0; c < 16; ++c) u->wch_host[c] = c < u->cfg.in_ch ? host_w[c] : 0.0f;
    UCHK(hipMemcpy(u->wch, u->wch_host, 64, hipMemcpyHostToDevice));
    return LBPF_OK;
}

lbpf_status lbpf_unet_forward(lbpf_unet* u, const float* in, float* out, int32_t n, int32_t h, int32_t w) {
    if (!u || !in || !out) return u ? ufail(u, LBPF_E_INVALID, "NULL buffer") : LBPF_E_INVALID;
    u->err.clear();
    if (lbpf_status s = check_dims(u, n, h, w)) return s;
    return forward(u, in, n, h, w, out);
}

lbpf_status lbpf_unet_loss_grad(lbpf_unet* u, const float* in, const float* target, int32_t n,
                                int32_t h, int32_t w, double* loss_host, float* grad_out) {
    if (!u || !in || !target) return u ? ufail(u, LBPF_E_INVALID, "NULL buffer") : LBPF_E_INVALID;
    u->err.clear();
    if (!u->grad) return ufail(u, LBPF_E_STATE, "created without training buffers (cfg.train = 0)");
    if (lbpf_status s = check_dims(u, n, h, w)) return s;
    if (lbpf_status s = forward(u, in, n, h, w, nullptr)) return s;
    UCHK(unet_predict_loss(in, u->head32, u->cfg.in_ch, nullptr, target, u->wch, u->gact[YH],
                           (long long)n * h * w, u->loss_part, kLossBlocks, u->stream));
    if (lbpf_status s = backward(u, n, h, w)) return s;
    if (grad_out) UCHK(hipMemcpyAsync(grad_out, u->grad, u->g.nparam * 4, hipMemcpyDeviceToDevice, u->stream));
    return loss_reduce(u, (long long)n * h * w, loss_host);
}

lbpf_status lbpf_unet_train_step(lbpf_unet* u, const float* in, const float* target, int32_t n,
                                 int32_t h, int32_t w, float lr, double* loss_host) {
    if (lbpf_status s = lbpf_unet_loss_grad(u, in, target, n, h, w, loss_host, nullptr)) return s;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    u->adam_t += 1;
    const float c1 = 1.0f / (1.0f - std::pow(b1, (float)u->adam_t));
    const float c2 = 1.0f / (1.0f - std::pow(b2, (float)u->adam_t));
    UCHK(unet_adam(u->w32, u->wbf, u->grad, u->adam_m, u->adam_v, u->g.nparam, lr, b1, b2, eps, c1, c2, u->stream));
    return LBPF_OK;
}

lbpf_status lbpf_unet_destroy(lbpf_unet* u) {
    delete u;
    return LBPF_OK;
}

const char* lbpf_unet_last_error(const lbpf_unet* u) { return u ? u->err.c_str() : g_unet_err.c_str(); }

lbpf_status lbpf_unet_conv_probe(const lbpf_unet_conv_desc* d, int32_t* variant, void* hip_stream) {
    if (!d || !d->wt || (!d->x && !d->xin) || (d->cl > 0 && !d->xl)) return LBPF_E_INVALID;
    if (d->n < 1 || d->h < 1 || d->w < 1 || d->cin < 1 || d->cout < 1 || d->cl < 0 || d->cl > d->cin)
        return LBPF_E_INVALID;
    if ((d->pred && !d->res) || (d->hw && !d->pred) || ((d->pred || d->hw) && (d->rc < 1 || d->rc > 16)))
        return LBPF_E_INVALID;
    ConvArgs a{};
    if (d->xin) {
        if (d->x || d->cl || d->xin_c < 1 || d->xin_c > 4) return LBPF_E_INVALID;
        a.xin = d->xin;
        a.xin_c = d->xin_c;
    } else {
        a.x = (const bf16*)d->x;
        a.xs = d->cin - d->cl;
        a.xo = 0;
    }
    a.xl = (const bf16*)d->xl;
    a.xls = d->cl;
    a.xlo = 0;
    a.Cl = d->cl;
    a.Cin = d->cin;
    a.w = (const bf16*)d->wt;
    a.bias = d->bias;
    a.y = (bf16*)d->y;
    a.ys = d->cout;
    a.yo = 0;
    a.yp = (bf16*)d->yp;
    a.yps = d->cout;
    a.ypo = 0;
    a.yf = d->yf;
    a.res = d->res;
    a.pred = d->pred;
    a.rc = d->rc;
    a.hw = (const bf16*)d->hw;
    a.hb = d->hb;
    a.Cout = d->cout;
    a.N = d->n;
    a.H = d->h;
    a.W = d->w;
    ConvPlan plan;
    if (unet_conv_plan(d->ks, a, &plan) != hipSuccess) return LBPF_E_INVALID;
    if (variant) {
        variant[0] = plan.first;
        variant[1] = plan.cot;
        variant[2] = plan.pfw;
    }
    return unet_conv(d->ks, d->relu != 0, a, (hipStream_t)hip_stream) == hipSuccess ? LBPF_OK : LBPF_E_HIP;
}

lbpf_status lbpf_unet_wgrad_probe(int32_t ks, const void* dy, const void* x, int32_t n, int32_t h,
                                  int32_t w, int32_t cin, int32_t cout, int32_t max_chunks,
                                  float* part, float* bpart, float* dw, float* db, void* hip_stream) {
    if (!dy || !x || !part || !bpart || !dw || !db || n < 1 || h < 1 || w < 1 || max_chunks < 1 ||
        (ks != 1 && ks != 3) || cin < 8 || cout < 8 || cin % 8 || cout % 8)
        return LBPF_E_INVALID;
    hipError_t e = unet_conv_wgrad(ks, (const bf16*)dy, cout, 0, cout, (const bf16*)x, cin, 0, cin, n, h, w,
                                   max_chunks, part, bpart, dw, db, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBPF_OK : LBPF_E_HIP;
}

lbpf_status lbpf_mfma_probe(int32_t k, const void* A, const void* B, float* D, void* hip_stream) {
    if (!A || !B || !D || (k != 16 && k != 32)) return LBPF_E_INVALID;
    hipError_t e = unet_mfma_probe(k == 32, (const bf16*)A, (const bf16*)B, D, (hipStream_t)hip_stream);
    return e == hipSuccess ? LBPF_OK : LBPF_E_HIP;
}

}  // extern "C"
