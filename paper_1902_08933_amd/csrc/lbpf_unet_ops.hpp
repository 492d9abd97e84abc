// Device operations of the surrogate network (kernels in lbpf_unet_kernels.hip), as the host
// side of the network (lbpf_unet.cpp) calls them. All activations are NHWC bf16 with a channel
// stride and offset, so a layer can read or write a slice of a concatenation buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbpf {

typedef uint16_t bf16;

// One convolution, KS x KS (1 or 3), stride 1, circular padding, on an N x H x W image:
//   v[p, co] = bias[co] + sum_{tap, ci} in[p + off(tap), ci] w[co, tap, ci],  optional ReLU.
// Input channels [0, Cl) are the nearest 2x upsampling of a half-resolution tensor xl
// (N x H/2 x W/2), channels [Cl, Cin) come from x at full resolution, so that the concat
// [up(a), b] of the decoder is never materialized (Cl = 0: x only).
// Outputs (each optional): y (bf16, post-activation), its 2x2 average pool yp (bf16,
// N x H/2 x W/2, the mean of the four bf16 values, H and W even), yf (FP32 [p][Cout]), and
// the prediction epilogue pred[p][c] = res[p][c] + v[p, c] for c < rc (FP32, rc channels).
// With hw set (a 3x3 layer whose Cout fits one workgroup, Cout <= 32), the epilogue instead
// applies a 1x1 head to the bf16-rounded outputs: pred[p][c] = res[p][c] + hb[c] +
// sum_ci hw[c][ci] bf16(v[p, ci]) for c < rc (hw: [>= rc][Cout] bf16, hb: FP32).
// Alignment: Cin, Cl, strides and offsets multiples of 8 (16-byte pieces); H, W even if Cl > 0.
struct ConvArgs {
    const bf16* x;
    int xs, xo;
    const bf16* xl;
    int xls, xlo, Cl;
    int Cin;
    const bf16* w;      // [Cout][KS*KS][Cin]
    const float* bias;  // Cout floats or NULL
    bf16* y;
    int ys, yo;
    bf16* yp;
    int yps, ypo;
    float* yf;
    const float* res;
    float* pred;
    int rc;
    const bf16* hw;
    const float* hb;
    // first layer: instead of x, the FP32 input NHWC with xin_c <= 4 fields (3x3 only); Cin is
    // then the channel stride of the weights
    const float* xin;
    int xin_c;
    int Cout, N, H, W;
};

// Kernel variant a convolution runs with: the first-layer kernel or the tiled one, its output
// channels per workgroup (16, 32, 64) and whether it prefetches the next chunk's weights.
struct ConvPlan {
    int first, cot, pfw;
};
hipError_t unet_conv_plan(int ks, const ConvArgs& a, ConvPlan* plan);
hipError_t unet_conv(int ks, bool relu, const ConvArgs& a, hipStream_t st);
// plain convolution (no upsampled part, bf16 output only)
hipError_t unet_conv_fwd(int ks, bool relu, const bf16* x, int xs, int xo, int Cin, const bf16* w,
                         const float* bias, bf16* y, int ys, int yo, int Cout, float* yf, int N,
                         int H, int W, hipStream_t st);
hipError_t unet_mfma_probe(int k32, const bf16* A, const bf16* B, float* D, hipStream_t st);
hipError_t unet_flip_weights(const bf16* w, bf16* wt, int Cout, int Cin, int taps, hipStream_t st);
// weight and bias gradients of a convolution (dw [Cout][KS*KS][Cin], db [Cout], FP32), from
// deterministic per-chunk partials: part and bpart hold at least max_chunks * Cout * KS*KS * Cin
// and max_chunks * Cout floats
hipError_t unet_conv_wgrad(int ks, const bf16* dy, int dys, int dyo, int Cout, const bf16* x, int xs,
                           int xo, int Cin, int N, int H, int W, int max_chunks, float* part,
                           float* bpart, float* dw, float* db, hipStream_t st);
// C channels (C, strides, offsets multiples of 8)
hipError_t unet_avgpool(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st);
hipError_t unet_avgpool_bwd_add(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st);
hipError_t unet_upsample(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st);
hipError_t unet_upsample_bwd(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st);
hipError_t unet_relu_bwd(bf16* g, int gs, int go, const bf16* a, int as, int ao, int C, long long npix, hipStream_t st);
hipError_t unet_pack_input(const float* in, int cin, bf16* x0, long long npix, hipStream_t st);
hipError_t unet_predict_loss(const float* in, const float* head, int cout, float* pred, const float* target,
                             const float* wch, bf16* dy, long long npix, double* part, int nblk, hipStream_t st);
hipError_t unet_adam(float* w, bf16* wb, const float* g, float* m, float* v, long long n, float lr, float b1,
                     float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t unet_to_bf16(const float* a, bf16* b, long long n, hipStream_t st);
hipError_t unet_bf16_to_f32(const bf16* b, float* a, long long n, hipStream_t st);

}  // namespace lbpf
