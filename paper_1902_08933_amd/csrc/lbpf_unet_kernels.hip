// HIP kernels of the learned surrogate (a small U-Net) for gfx950: BF16 storage of weights and
// activations, FP32 accumulation on MFMA (v_mfma_f32_16x16x16_bf16), NHWC layout, circular
// padding (the flow fields are periodic).
//
// MFMA operand layout used throughout (one wave, 64 lanes, lane = l):
//   A (16 x 16, row i, column k): lane i + 16 * (k / 4) holds A[i][k] in element k % 4
//   B (16 x 16, row k, column j): lane j + 16 * (k / 4) holds B[k][j] in element k % 4
//   D (16 x 16 FP32):             lane j + 16 * (i / 4) holds D[i][j] in element i % 4
// (checked bit-exactly against integer arithmetic by mfma_probe_kernel's test).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>

#include "lbpf_unet_ops.hpp"

namespace lbpf {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ bf16 f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 b) { return __uint_as_float((uint32_t)b << 16); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// two FP32 values as packed bf16 (round to nearest even as f2bf, one instruction)
__device__ __forceinline__ uint32_t pack_bf2(float x, float y) {
    const bf16x2_t v = {(__bf16)x, (__bf16)y};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float4_t mfma16(short4_t a, short4_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef short short8_t __attribute__((ext_vector_type(8)));

// gfx950 double-K form: A 16 x 32, B 32 x 16; lane i + 16 * (k / 8) holds A[i][k] in element
// k % 8 (B likewise with the column), D as for the 16 x 16 x 16 form
__device__ __forceinline__ float4_t mfma32(short8_t a, short8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ short4_t load4(const bf16* p) {
    return *reinterpret_cast<const short4_t*>(p);
}

// One 16x16x16 product of row-major A (16x16) and B (16x16) bf16 into D (16x16 FP32).
__global__ void mfma_probe_kernel(const bf16* __restrict__ A, const bf16* __restrict__ B,
                                  float* __restrict__ D) {
    const int l = threadIdx.x;
    short4_t a, b;
    for (int e = 0; e < 4; ++e) {
        a[e] = (short)A[(l % 16) * 16 + 4 * (l / 16) + e];
        b[e] = (short)B[(4 * (l / 16) + e) * 16 + l % 16];
    }
    float4_t d = {0.f, 0.f, 0.f, 0.f};
    d = mfma16(a, b, d);
    for (int e = 0; e < 4; ++e) D[(4 * (l / 16) + e) * 16 + l % 16] = d[e];
}

// One 16x16x32 product (row-major A 16x32, B 32x16 bf16) into D (16x16 FP32).
__global__ void mfma32_probe_kernel(const bf16* __restrict__ A, const bf16* __restrict__ B,
                                    float* __restrict__ D) {
    const int l = threadIdx.x;
    short8_t a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = (short)A[(l % 16) * 32 + 8 * (l / 16) + e];
        b[e] = (short)B[(8 * (l / 16) + e) * 16 + l % 16];
    }
    float4_t d = {0.f, 0.f, 0.f, 0.f};
    d = mfma32(a, b, d);
    for (int e = 0; e < 4; ++e) D[(4 * (l / 16) + e) * 16 + l % 16] = d[e];
}

// Convolution (contract in lbpf_unet_ops.hpp) as an implicit GEMM on MFMA: M = pixels,
// N = output channels, K = KS*KS*Cin. A workgroup of 4 waves computes a tile of TR x TC
// pixels of one image for COT output channels; wave w owns rows 4w .. 4w+3 of the tile, i.e.
// four 16-pixel A fragments, so every B fragment read from LDS feeds four MFMAs. Per chunk of
// 32 input channels the input patch (with its KS-1 halo, circular) and the weights of the COT
// channels are staged in LDS (rows padded to 40 bf16 so that the 16 lanes of a fragment read hit
// 16 different bank groups); each tap is then a 16x16x32 MFMA per (row fragment, 16 channels).
// The next chunk is fetched into registers while the current one is multiplied. Channels below
// Cl are read from the half-resolution tensor at (y/2, x/2): the nearest 2x upsampling fused
// into the load. Pixels beyond a ragged image edge are computed from wrapped data and not
// stored. The bf16 output leaves through LDS as 16-byte stores, and so does its 2x2 average
// pool when asked for (tiles start at even coordinates, so every pool window is inside one).
constexpr int kConvTR = 16, kConvTC = 16, kConvCK = 32, kConvCKP = 40;

template <int KS, int COT>
constexpr int conv_lds_elems() {
    constexpr int PR = kConvTR + KS - 1, PC = kConvTC + KS - 1;
    constexpr int in = PR * PC * kConvCKP + COT * KS * KS * kConvCKP;
    // output tile (bf16, padded rows) followed by the fused head's FP32 outputs [pixel][16]
    constexpr int out = kConvTR * kConvTC * (COT + 8) + kConvTR * kConvTC * 16 * 2;
    return in > out ? in : out;
}

__device__ __forceinline__ int wrap_coord(int v, int m) {
    if ((unsigned)v < (unsigned)m) return v;
    const int r = v % m;
    return r < 0 ? r + m : r;
}

// Epilogue shared by the convolution kernels: bias, activation and the outputs of ConvArgs
// (bf16 tile through LDS, its 2x2 pool, FP32 copy, prediction, fused head) for a tile of
// TR x TC pixels at (tx0, ty0) of image n and output channels co0 .. co0 + COT - 1, from the
// accumulators of the 4 waves (wave w: rows MF w .. MF w + MF - 1). The caller has finished
// with its LDS; s_o is the start of the workgroup's LDS.
template <bool RELU, int COT, int MF>
__device__ __forceinline__ void conv_epilogue(const ConvArgs& a, const float4_t (&acc)[MF][COT / 16],
                                              bf16* s_o, int tx0, int ty0, int n, int co0) {
    constexpr int TR = kConvTR, TC = kConvTC, NF = COT / 16, COTP = COT + 8;
    static_assert(TR == 4 * MF, "four waves of MF rows");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, m = lane & 15;
    const int H = a.H, W = a.W, Cout = a.Cout;
    static_assert(TR * TC == 256, "the fused head's residual is one pixel per thread");
    // the fused head's residual (4 fields) is read now, so that its latency overlaps the
    // output tile's stores and barriers
    float4 res4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int rpy = ty0 + tid / TC, rpx = tx0 + tid % TC;
    const bool res_vec = a.hw && a.rc == 4 && rpy < H && rpx < W;
    if (res_vec) res4 = *reinterpret_cast<const float4*>(a.res + ((size_t)(n * H + rpy) * W + rpx) * 4);
    // D fragment: lane (16 * g + c) holds pixels 4g .. 4g+3 of the row, channel c
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        const int co = co0 + 16 * j + m;
        const float bb = (a.bias && co < Cout) ? a.bias[co] : 0.0f;
#pragma unroll
        for (int f = 0; f < MF; ++f) {
            const int py = wave * MF + f, yy = ty0 + py;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int px = 4 * (lane >> 4) + e, xx = tx0 + px;
                float v = acc[f][j][e] + bb;
                if (RELU) v = fmaxf(v, 0.0f);
                if (a.y || a.yp || a.hw) s_o[(py * TC + px) * COTP + 16 * j + m] = f2bf(v);
                if (yy < H && xx < W && co < Cout) {
                    const size_t p = (size_t)(n * H + yy) * W + xx;
                    if (a.yf) a.yf[p * Cout + co] = v;
                    if (a.pred && !a.hw && co < a.rc) a.pred[p * a.rc + co] = a.res[p * a.rc + co] + v;
                }
            }
        }
    }
    if (!a.y && !a.yp && !a.hw) return;
    __syncthreads();
    if (a.hw) {
        // fused 1x1 head on the bf16 outputs of this tile (all Cout <= 32 channels are in s_o):
        // per 16-pixel row one 16x16x32 MFMA, A = pixels x channels, B = channels x head outputs
        const int g = lane >> 4;
        short8_t hwf = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (m < a.rc && 8 * g + e < Cout) hwf[e] = (short)a.hw[m * Cout + 8 * g + e];
        const float hbias = (a.hb && m < a.rc) ? a.hb[m] : 0.0f;
        float* s_h = reinterpret_cast<float*>(s_o + TR * TC * COTP);
#pragma unroll
        for (int f = 0; f < MF; ++f) {
            const int py = wave * MF + f, yy = ty0 + py;
            short8_t av = {0, 0, 0, 0, 0, 0, 0, 0};
            if (8 * g < Cout) av = *reinterpret_cast<const short8_t*>(s_o + (py * TC + m) * COTP + 8 * g);
            const float4_t d = mfma32(av, hwf, float4_t{0.f, 0.f, 0.f, 0.f});
            // D: lane (m + 16 g) holds pixels 4g .. 4g+3 of the row, head output m
#pragma unroll
            for (int e = 0; e < 4; ++e) s_h[(py * TC + 4 * g + e) * 16 + m] = d[e] + hbias;
            (void)yy;
        }
        __syncthreads();
        // prediction = input + head, one pixel per thread with 16-byte accesses for 4 fields
        for (int pix = tid; pix < TR * TC; pix += 256) {
            const int yy = ty0 + pix / TC, xx = tx0 + pix % TC;
            if (yy >= H || xx >= W) continue;
            const size_t p = (size_t)(n * H + yy) * W + xx;
            if (a.rc == 4) {
                const float4 r = res4;  // pix == tid: this thread's prefetched residual
                const float4 hv = *reinterpret_cast<const float4*>(s_h + pix * 16);
                *reinterpret_cast<float4*>(a.pred + p * 4) = make_float4(r.x + hv.x, r.y + hv.y, r.z + hv.z, r.w + hv.w);
            } else {
                for (int c = 0; c < a.rc; ++c) a.pred[p * a.rc + c] = a.res[p * a.rc + c] + s_h[pix * 16 + c];
            }
        }
    }
    if (a.y) {
        for (int piece = tid; piece < TR * TC * (COT / 8); piece += 256) {
            const int q = piece % (COT / 8), pix = piece / (COT / 8);
            const int yy = ty0 + pix / TC, xx = tx0 + pix % TC, co = co0 + 8 * q;
            if (yy < H && xx < W && co < Cout)
                *reinterpret_cast<short8_t*>(a.y + ((size_t)(n * H + yy) * W + xx) * a.ys + a.yo + co) =
                    *reinterpret_cast<const short8_t*>(s_o + pix * COTP + 8 * q);
        }
    }
    if (a.yp) {
        const int Hp = H >> 1, Wp = W >> 1;
        for (int piece = tid; piece < (TR / 2) * (TC / 2) * (COT / 8); piece += 256) {
            const int q = piece % (COT / 8), pix = piece / (COT / 8);
            const int py = pix / (TC / 2), px = pix % (TC / 2);
            const int yy = (ty0 >> 1) + py, xx = (tx0 >> 1) + px, co = co0 + 8 * q;
            if (yy >= Hp || xx >= Wp || co >= Cout) continue;
            const bf16* o = s_o + ((2 * py) * TC + 2 * px) * COTP + 8 * q;
            const short8_t v0 = *reinterpret_cast<const short8_t*>(o);
            const short8_t v1 = *reinterpret_cast<const short8_t*>(o + COTP);
            const short8_t v2 = *reinterpret_cast<const short8_t*>(o + TC * COTP);
            const short8_t v3 = *reinterpret_cast<const short8_t*>(o + (TC + 1) * COTP);
            short8_t r;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                r[k] = (short)f2bf(0.25f * (bf2f((bf16)v0[k]) + bf2f((bf16)v1[k]) + bf2f((bf16)v2[k]) +
                                            bf2f((bf16)v3[k])));
            *reinterpret_cast<short8_t*>(a.yp + ((size_t)(n * Hp + yy) * Wp + xx) * a.yps + a.ypo + co) = r;
        }
    }
}

// First layer of the network: the input is FP32 NHWC with xin_c <= 4 fields. The K dimension of
// the implicit GEMM is ordered (tap, field), so the 9 x 4 = 36 products of a 3x3 convolution
// fill two 16x16x32 MFMA steps (zero beyond tap 8) instead of one step per tap with the fields
// padded to 32 channels. The input patch is converted to bf16 into LDS (8 bytes per pixel);
// the weights of the workgroup's channels stay in registers.
template <bool RELU, int COT>
__global__ __launch_bounds__(256, 2) void conv_first_kernel(const ConvArgs a) {
    constexpr int TR = kConvTR, TC = kConvTC, PR = TR + 2, PC = TC + 2;
    constexpr int MF = TR / 4, NF = COT / 16;
    extern __shared__ __attribute__((aligned(16))) bf16 conv_lds[];
    bf16* s_x = conv_lds;  // [PR * PC][4]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, m = lane & 15, g = lane >> 4;
    const int H = a.H, W = a.W, Cout = a.Cout, cin = a.xin_c, wcin = a.Cin;
    const int tiles_x = (W + TC - 1) / TC, tiles_y = (H + TR - 1) / TR;
    const int tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TC, ty0 = ((tile / tiles_x) % tiles_y) * TR;
    const int n = tile / (tiles_x * tiles_y);
    const int co0 = blockIdx.y * COT;
    // the workgroup's weights, fields 0..3 of every (channel, tap), staged once in LDS as
    // [COT][9][4] bf16 (zero beyond Cout and beyond the input's fields)
    bf16* s_wf = conv_lds + PR * PC * 4;
    for (int r = tid; r < COT * 9; r += 256) {
        const int co = co0 + r / 9, t = r % 9;
        short4_t v = {0, 0, 0, 0};
        if (co < Cout) {
            const bf16* src = a.w + ((size_t)co * 9 + t) * wcin;
            if (wcin % 4 == 0 && cin == 4 && (reinterpret_cast<uintptr_t>(a.w) & 7) == 0) {
                v = *reinterpret_cast<const short4_t*>(src);
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < cin) v[c] = (short)src[c];
            }
        }
        *reinterpret_cast<short4_t*>(s_wf + r * 4) = v;
    }
    const bool vec_in = cin == 4 && (reinterpret_cast<uintptr_t>(a.xin) & 15) == 0;
    for (int pix = tid; pix < PR * PC; pix += 256) {
        const int sy = wrap_coord(ty0 + pix / PC - 1, H), sx = wrap_coord(tx0 + pix % PC - 1, W);
        const float* src = a.xin + ((size_t)(n * H + sy) * W + sx) * cin;
        short4_t v = {0, 0, 0, 0};
        if (vec_in) {
            const float4 f = *reinterpret_cast<const float4*>(src);
            v = {(short)f2bf(f.x), (short)f2bf(f.y), (short)f2bf(f.z), (short)f2bf(f.w)};
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < cin) v[c] = (short)f2bf(src[c]);
        }
        *reinterpret_cast<short4_t*>(s_x + pix * 4) = v;
    }
    __syncthreads();
    // B[k][co] with k = 4 tap + field: lane (m + 16 g) holds k = 32 s + 8 g + e, i.e. taps
    // 8 s + 2 g (e < 4) and 8 s + 2 g + 1 (e >= 4), field e % 4
    short8_t b[2][NF];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            const int r = (16 * j + m) * 9, t0 = 8 * st + 2 * g;
            const short4_t w0 = t0 < 9 ? *reinterpret_cast<const short4_t*>(s_wf + (r + t0) * 4) : short4_t{0, 0, 0, 0};
            const short4_t w1 = t0 + 1 < 9 ? *reinterpret_cast<const short4_t*>(s_wf + (r + t0 + 1) * 4)
                                           : short4_t{0, 0, 0, 0};
            b[st][j] = short8_t{w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
        }
    float4_t acc[MF][NF];
#pragma unroll
    for (int f = 0; f < MF; ++f)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[f][j] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int row = wave * MF + f;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const int t0 = 8 * st + 2 * g, t1 = t0 + 1;
            short4_t x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
            if (t0 < 9) x0 = *reinterpret_cast<const short4_t*>(s_x + ((row + t0 / 3) * PC + m + t0 % 3) * 4);
            if (t1 < 9) x1 = *reinterpret_cast<const short4_t*>(s_x + ((row + t1 / 3) * PC + m + t1 % 3) * 4);
            const short8_t av = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
#pragma unroll
            for (int j = 0; j < NF; ++j) acc[f][j] = mfma32(av, b[st][j], acc[f][j]);
        }
    }
    __syncthreads();  // LDS is reused for the output tile
    conv_epilogue<RELU, COT, MF>(a, acc, conv_lds, tx0, ty0, n, co0);
}

// First layer, persistent (inference: 4 FP32 fields in, 32 output channels, the bf16 output and
// its 2x2 pool out, images of whole 16 x 16 tiles): the arithmetic of conv_first_kernel, with
// the weights staged and turned into B operands once per workgroup, and the next tile's input
// patch loaded into registers while the current one is computed and stored. Three separate LDS
// areas (output tile, patch, weights), so that a tile's patch can be written while nothing reads
// it; fence-free barriers, because __syncthreads would also wait for the prefetched patch.
template <bool RELU>
__global__ __launch_bounds__(256) void conv_first_loop_kernel(const ConvArgs a, int ntiles) {
    constexpr int TR = kConvTR, TC = kConvTC, PR = TR + 2, PC = TC + 2, C = 32, NF = C / 16, MF = TR / 4;
    constexpr int NPIX = PR * PC, COTP = C + 8;
    static_assert(NPIX > 256 && NPIX <= 512, "two patch pixels per thread at most");
    __shared__ __attribute__((aligned(16))) bf16 s_o[TR * TC * COTP];
    __shared__ __attribute__((aligned(16))) bf16 s_x[NPIX * 4];
    __shared__ __attribute__((aligned(16))) bf16 s_wf[C * 9 * 4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, m = lane & 15, g = lane >> 4;
    const int H = a.H, W = a.W, wcin = a.Cin;
    const int tiles_x = W / TC, tiles_y = H / TR;
    for (int r = tid; r < C * 9; r += 256) {
        const bf16* src = a.w + ((size_t)(r / 9) * 9 + r % 9) * wcin;
        *reinterpret_cast<short4_t*>(s_wf + r * 4) = *reinterpret_cast<const short4_t*>(src);
    }
    float bb[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) bb[j] = a.bias ? a.bias[16 * j + m] : 0.0f;
    __syncthreads();
    // B operands as in conv_first_kernel: lane (m + 16 g) holds k = 32 s + 8 g + e, i.e. taps
    // 8 s + 2 g (e < 4) and 8 s + 2 g + 1 (e >= 4), field e % 4, of channel 16 j + m
    short8_t b[2][NF];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            const int r = (16 * j + m) * 9, t0 = 8 * st + 2 * g;
            const short4_t w0 = t0 < 9 ? *reinterpret_cast<const short4_t*>(s_wf + (r + t0) * 4) : short4_t{0, 0, 0, 0};
            const short4_t w1 = t0 + 1 < 9 ? *reinterpret_cast<const short4_t*>(s_wf + (r + t0 + 1) * 4)
                                           : short4_t{0, 0, 0, 0};
            b[st][j] = short8_t{w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
        }
    // the patch of a tile (pixels tid and tid + 256 of its 18 x 18, circular), into registers
    float4 px0, px1;
    auto fetch = [&](int tile) __attribute__((always_inline)) {
        const int tx0 = (tile % tiles_x) * TC, ty0 = ((tile / tiles_x) % tiles_y) * TR, n = tile / (tiles_x * tiles_y);
        const int p1 = tid + 256 < NPIX ? tid + 256 : NPIX - 1;
        const int y0 = wrap_coord(ty0 + tid / PC - 1, H), x0 = wrap_coord(tx0 + tid % PC - 1, W);
        const int y1 = wrap_coord(ty0 + p1 / PC - 1, H), x1 = wrap_coord(tx0 + p1 % PC - 1, W);
        px0 = *reinterpret_cast<const float4*>(a.xin + ((size_t)(n * H + y0) * W + x0) * 4);
        px1 = *reinterpret_cast<const float4*>(a.xin + ((size_t)(n * H + y1) * W + x1) * 4);
    };
    auto put = [&](int pix, const float4& f) __attribute__((always_inline)) {
        *reinterpret_cast<uint2*>(s_x + pix * 4) = make_uint2(pack_bf2(f.x, f.y), pack_bf2(f.z, f.w));
    };
    int tile = blockIdx.x;
    if (tile < ntiles) fetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int tx0 = (tile % tiles_x) * TC, ty0 = ((tile / tiles_x) % tiles_y) * TR, n = tile / (tiles_x * tiles_y);
        put(tid, px0);
        if (tid + 256 < NPIX) put(tid + 256, px1);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // the next tile's patch (this one's again after the last tile)
        const int nt = tile + (int)gridDim.x;
        fetch(nt < ntiles ? nt : tile);
        float4_t acc[MF][NF];
#pragma unroll
        for (int f = 0; f < MF; ++f) {
            const int row = wave * MF + f;
#pragma unroll
            for (int j = 0; j < NF; ++j) acc[f][j] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const int t0 = 8 * st + 2 * g, t1 = t0 + 1;
                short4_t x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
                if (t0 < 9) x0 = *reinterpret_cast<const short4_t*>(s_x + ((row + t0 / 3) * PC + m + t0 % 3) * 4);
                if (t1 < 9) x1 = *reinterpret_cast<const short4_t*>(s_x + ((row + t1 / 3) * PC + m + t1 % 3) * 4);
                const short8_t av = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
#pragma unroll
                for (int j = 0; j < NF; ++j) acc[f][j] = mfma32(av, b[st][j], acc[f][j]);
            }
        }
        // D fragment: lane (16 g + c) holds pixels 4g .. 4g+3 of the row, channel 16 j + c
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int f = 0; f < MF; ++f)
#pragma unroll
                for (int e = 0; e < 4; e += 2) {
                    float v0 = acc[f][j][e] + bb[j], v1 = acc[f][j][e + 1] + bb[j];
                    if (RELU) v0 = fmaxf(v0, 0.0f), v1 = fmaxf(v1, 0.0f);
                    const uint32_t pk = pack_bf2(v0, v1);
                    s_o[((wave * MF + f) * TC + 4 * g + e) * COTP + 16 * j + m] = (bf16)(pk & 0xffff);
                    s_o[((wave * MF + f) * TC + 4 * g + e + 1) * COTP + 16 * j + m] = (bf16)(pk >> 16);
                }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (a.y) {
#pragma unroll
            for (int k = 0; k < TR * TC * (C / 8) / 256; ++k) {
                const int piece = tid + 256 * k, q = piece % (C / 8), pix = piece / (C / 8);
                const int yy = ty0 + pix / TC, xx = tx0 + pix % TC;
                *reinterpret_cast<short8_t*>(a.y + ((size_t)(n * H + yy) * W + xx) * a.ys + a.yo + 8 * q) =
                    *reinterpret_cast<const short8_t*>(s_o + pix * COTP + 8 * q);
            }
        }
        if (a.yp) {
            // 2x2 mean of the bf16 outputs, summed (0,0), (0,1), (1,0), (1,1)
            static_assert((TR / 2) * (TC / 2) * (C / 8) == 256, "one pooled piece per thread");
            const int q = tid % (C / 8), pix = tid / (C / 8), py = pix / (TC / 2), px = pix % (TC / 2);
            const int Hp = H >> 1, Wp = W >> 1, yy = (ty0 >> 1) + py, xx = (tx0 >> 1) + px;
            const bf16* o = s_o + ((2 * py) * TC + 2 * px) * COTP + 8 * q;
            const short8_t v0 = *reinterpret_cast<const short8_t*>(o);
            const short8_t v1 = *reinterpret_cast<const short8_t*>(o + COTP);
            const short8_t v2 = *reinterpret_cast<const short8_t*>(o + TC * COTP);
            const short8_t v3 = *reinterpret_cast<const short8_t*>(o + (TC + 1) * COTP);
            uint32_t r[4];
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                const float s0 = bf2f((bf16)v0[k]) + bf2f((bf16)v1[k]) + bf2f((bf16)v2[k]) + bf2f((bf16)v3[k]);
                const float s1 = bf2f((bf16)v0[k + 1]) + bf2f((bf16)v1[k + 1]) + bf2f((bf16)v2[k + 1]) +
                                 bf2f((bf16)v3[k + 1]);
                r[k / 2] = pack_bf2(0.25f * s0, 0.25f * s1);
            }
            *reinterpret_cast<uint4*>(a.yp + ((size_t)(n * Hp + yy) * Wp + xx) * a.yps + a.ypo + 8 * q) =
                make_uint4(r[0], r[1], r[2], r[3]);
        }
    }
}

// PFW: the next chunk's weights are fetched into registers with the patch, so that no global
// latency is exposed when a chunk is published. It costs registers: COT = 32 then runs at two
// workgroups per CU instead of three (taken when the grid is too small to fill three), and
// COT = 64 at the register limit (a few spills) instead of loading its weights from L2 while
// publishing (measured faster with the prefetch).
template <int KS, bool RELU, int COT, bool PFW>
__global__ __launch_bounds__(256, (COT <= 32 && !PFW ? 3 : 2)) void conv_tile_kernel(const ConvArgs a) {
    constexpr int TR = kConvTR, TC = kConvTC, CK = kConvCK, CKP = kConvCKP;
    constexpr int HALO = KS - 1, PR = TR + HALO, PC = TC + HALO, T = KS * KS;
    constexpr int PIECES = CK / 8;                  // 16-byte pieces per pixel and chunk
    constexpr int NPATCH = PR * PC * PIECES;
    constexpr int NWT = COT * T * PIECES;
    constexpr int PP = (NPATCH + 255) / 256, PW = (NWT + 255) / 256;
    constexpr int MF = TR / 4, NF = COT / 16;
    extern __shared__ __attribute__((aligned(16))) bf16 conv_lds[];
    bf16* s_x = conv_lds;
    bf16* s_w = conv_lds + PR * PC * CKP;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int H = a.H, W = a.W, Cin = a.Cin, Cl = a.Cl, Cout = a.Cout;
    const int tiles_x = (W + TC - 1) / TC, tiles_y = (H + TR - 1) / TR;
    const int tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TC, ty0 = ((tile / tiles_x) % tiles_y) * TR;
    const int n = tile / (tiles_x * tiles_y);
    const int co0 = blockIdx.y * COT;
    const int h0 = HALO / 2, Hl = H >> 1, Wl = W >> 1;

    constexpr int PWR = PFW ? PW : 1;
    short8_t rp[PP], rw[PWR];
    auto fetch_w = [&](int i, int kc) {
        const int piece = tid + 256 * i;
        short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
        const int q = piece % PIECES, r = piece / PIECES;
        const int co = co0 + r / T, ci = kc + 8 * q;
        if (piece < NWT && co < Cout && ci < Cin)
            v = *reinterpret_cast<const short8_t*>(a.w + ((size_t)co * T + r % T) * Cin + ci);
        return v;
    };
    auto fetch = [&](int kc) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int piece = tid + 256 * i;
            short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (piece < NPATCH) {
                const int q = piece % PIECES, pix = piece / PIECES;
                const int sy = wrap_coord(ty0 + pix / PC - h0, H), sx = wrap_coord(tx0 + pix % PC - h0, W);
                const int ci = kc + 8 * q;
                if (ci < Cl)
                    v = *reinterpret_cast<const short8_t*>(
                        a.xl + ((size_t)(n * Hl + (sy >> 1)) * Wl + (sx >> 1)) * a.xls + a.xlo + ci);
                else if (ci < Cin)
                    v = *reinterpret_cast<const short8_t*>(
                        a.x + ((size_t)(n * H + sy) * W + sx) * a.xs + a.xo + (ci - Cl));
            }
            rp[i] = v;
        }
        if (PFW) {
#pragma unroll
            for (int i = 0; i < PWR; ++i) rw[i] = fetch_w(i, kc);
        }
    };
    // the patch (and with PFW the weights) come from the registers fetched during the previous
    // chunk; otherwise the weights (a few tens of KB, shared by every workgroup and resident in
    // L2) are loaded here, so that no registers hold them across the MFMA loop
    auto publish = [&](int kc) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int piece = tid + 256 * i;
            if (piece < NPATCH)
                *reinterpret_cast<short8_t*>(s_x + (piece / PIECES) * CKP + 8 * (piece % PIECES)) = rp[i];
        }
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int piece = tid + 256 * i;
            if (piece < NWT)
                *reinterpret_cast<short8_t*>(s_w + (piece / PIECES) * CKP + 8 * (piece % PIECES)) =
                    PFW ? rw[PFW ? i : 0] : fetch_w(i, kc);
        }
    };

    float4_t acc[MF][NF];
#pragma unroll
    for (int f = 0; f < MF; ++f)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[f][j] = {0.f, 0.f, 0.f, 0.f};
    const int m = lane & 15, kq = 8 * (lane >> 4);
    fetch(0);
    for (int kc = 0; kc < Cin; kc += CK) {
        __syncthreads();
        publish(kc);
        __syncthreads();
        if (kc + CK < Cin) fetch(kc + CK);
#pragma unroll
        for (int tap = 0; tap < T; ++tap) {
            const int dy = KS == 3 ? tap / 3 - 1 : 0, dx = KS == 3 ? tap % 3 - 1 : 0;
            short8_t b[NF];
#pragma unroll
            for (int j = 0; j < NF; ++j)
                b[j] = *reinterpret_cast<const short8_t*>(s_w + ((16 * j + m) * T + tap) * CKP + kq);
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const int row = wave * MF + f;
                const short8_t av = *reinterpret_cast<const short8_t*>(
                    s_x + ((row + dy + h0) * PC + (m + dx + h0)) * CKP + kq);
#pragma unroll
                for (int j = 0; j < NF; ++j) acc[f][j] = mfma32(av, b[j], acc[f][j]);
            }
        }
    }

    __syncthreads();  // LDS is reused for the output tile
    conv_epilogue<RELU, COT, MF>(a, acc, conv_lds, tx0, ty0, n, co0);
}

// 3x3 convolution in wave-row form, for Cin, Cl and Cout multiples of 32. Persistent
// workgroups of 4 waves walk work items (an image tile of 16 rows x 16 PX columns and 32 CG
// output channels, PX = 4 / CG) in XCD bands: workgroup b runs on XCD b % 8 and takes items of
// the band of that XCD, so that neighbouring tiles, which share halo pixels, share an L2.
// Wave w owns 16 rows x 16 columns (column block w / CG) of the item for 32 output channels
// (group w % CG); the image is at least one patch in size (H >= 18, W >= 16 PX + 2), so patch
// coordinates wrap by at most one period. Per chunk of 32 input channels (one step of the pipeline):
//  - the chunk's weights of the wave's 32 channels for all 9 taps sit in registers (18 MFMA
//    operands); once a column of taps is done its registers take the next step's weights;
//  - the input patch (18 rows x 16 PX + 2 columns, circular) is in LDS, double-buffered; its
//    pieces are loaded into registers between the MFMAs of the previous step and stored at
//    the start of the step;
//  - the wave reads each patch row once per horizontal tap dx and applies it to the up to three
//    output rows it reaches (vertical taps), two 16-channel MFMAs each: 54 fragment reads for
//    288 MFMAs (16x16x32) per chunk.
// The MFMA computes D = weights (16 channels x 32 K) x patch (32 K x 16 pixels), so lane
// j + 16 q of an accumulator holds channels 4q .. 4q+3 of pixel j: the epilogue (bias, ReLU,
// bf16, the 2x2 pool by a lane swap, FP32 copy, prediction) stores from registers, and the
// fused 1x1 head is one more MFMA whose operand is the wave's own bf16 outputs. One wave per
// SIMD: a wave holds 512 registers (accumulators 128, weights 72), so nothing is spilled.
// LDS: pixel p of the patch (row-major, PCOL columns) takes 64 bytes; its 16-byte piece k holds
// the chunk's channels 8 (k ^ ((col >> 1) & 3)) .. +7, col = p % PCOL. The swizzle puts any 8
// consecutive pixels' pieces of one channel group on 8 different 4-bank groups, so the
// fragment reads (16 consecutive pixels of a row) are conflict-free without padding; each store
// of staged pieces writes 64 consecutive ones.
constexpr int kWvRows = 16;      // rows of a work item
constexpr int kWvRowsHalf = 8;   // rows of a work item on small grids (128 channels per item)
constexpr int kWaveMaxCout = 512;  // output channels of the wave-row kernel at most

template <int CG, int RW = kWvRows>
struct WaveConvGeom {
    static constexpr int PX = 4 / CG;                 // 16-column blocks of a work item
    static constexpr int PCOL = 16 * PX + 2;          // patch columns, with the halo
    static constexpr int PROWS = RW + 2;              // patch rows
    static constexpr int NPIECE = PROWS * PCOL * 4;   // 16-byte pieces of one chunk's patch
    static constexpr int NBW = (NPIECE + 255) / 256;  // 64-piece load blocks per wave (one
                                                      // instruction each, every wave the same)
    static constexpr int BUF_BYTES = NPIECE * 16;     // a patch buffer (padding lanes of the
                                                      // last load block rewrite its last piece)
    static constexpr int LDS_BYTES = 2 * BUF_BYTES + kWaveMaxCout * 4;  // two buffers, the bias
};

// the two bf16 halves of a packed pair as FP32
__device__ __forceinline__ float bf_lo(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float bf_hi(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }
// value of lane l ^ 1
__device__ __forceinline__ float swap_lane_pair(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
// v mod m for v in [-m, 2m)
__device__ __forceinline__ int wrap_near(int v, int m) {
    return v < 0 ? v + m : (v >= m ? v - m : v);
}

// Outputs of the wave-row kernel, fixed at compile time to keep the code of each variant small:
// any of ConvArgs' outputs (checked at run time), y only, y and its pool, or the fused head
// with a 4-field prediction.
enum WaveOut { kOutAny = 0, kOutY = 1, kOutYPool = 2, kOutHead = 3 };

template <int CG, bool RELU, int OUT, int RW = kWvRows>
__global__ __launch_bounds__(256, 1) void conv3_wave_kernel(const ConvArgs a, int total_items) {
    using G = WaveConvGeom<CG, RW>;
    constexpr int PX = G::PX, PCOL = G::PCOL, NPIECE = G::NPIECE, NBW = G::NBW, R = RW;
    static_assert(R % 4 == 0, "whole groups of 4 rows (the head's residual, the pool)");
    extern __shared__ __attribute__((aligned(16))) uint8_t wconv_lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int jl = lane & 15, q = lane >> 4;
    const int cg = wave % CG, pxb = wave / CG;
    const int H = a.H, W = a.W, Cin = a.Cin, Cl = a.Cl, Cout = a.Cout;
    const int Hl = H >> 1, Wl = W >> 1;
    const int tiles_x = (W + 16 * PX - 1) / (16 * PX), tiles_y = (H + R - 1) / R;
    const int groups = Cout / (32 * CG);
    // the band of work items of this workgroup's XCD (the grid has at least 8 workgroups)
    const int nwg = gridDim.x, xcd = blockIdx.x % 8, loc = blockIdx.x / 8;
    const int nloc = (nwg - xcd + 7) / 8;
    const int band1 = (int)((long long)total_items * (xcd + 1) / 8);
    int item = (int)((long long)total_items * xcd / 8) + loc;
    if (item >= band1) return;
    // the bias of every output channel, behind the two patch buffers (the first barrier
    // publishes it)
    float* s_bias = reinterpret_cast<float*>(wconv_lds + 2 * G::BUF_BYTES);

    // origin of the item whose patch is being loaded
    int l_n = 0, l_ty0 = 0, l_tx0 = 0;
    auto plan_loads = [&](int it) __attribute__((always_inline)) {
        int t = it / groups;
        l_tx0 = (t % tiles_x) * 16 * PX;
        t /= tiles_x;
        l_ty0 = (t % tiles_y) * R;
        l_n = t / tiles_y;
    };
    // Load blocks. The patch in LDS is [patch row][column][4 slots of 16 bytes], slot g of
    // column c holding channel group g ^ ((c >> 1) & 3). Load block w = 4 i + wave (64 lanes,
    // 16 bytes each): the first REG blocks are row segments, patch row w / BPR, columns
    // 16 (w % BPR) .. +15, lane l taking column 16 (w % BPR) + l / 4, slot l % 4, so that a
    // block's LDS slots are contiguous and its patch row is uniform; the last two columns of
    // every row (8 pieces a row) follow in LFB blocks, piece t = 64 (w - REG) + lane at row
    // t / 8, column 16 PX + (t % 8) / 4, slot t % 4 (past the end: the last piece again).
    constexpr int BPR = PX, REG = G::PROWS * BPR, LEFTN = G::PROWS * 8, LFB = (LEFTN + 63) / 64;
    static_assert(REG + LFB <= 4 * NBW, "every piece in a load block");
    // block i is a row segment on every wave: its row is uniform and its column (b = wave % BPR,
    // since BPR divides 4) is the same in every such block of the wave
    auto all_rows = [](int i) constexpr { return 4 * i + 3 < REG; };
    const int rb = wave % BPR;
    const int r_col = 16 * rb + (lane >> 2), r_gs = lane & 3, r_gg = r_gs ^ ((lane >> 3) & 3);
    // any block: the lane's patch row, column and slot (uniform branch on the block)
    auto piece = [&](int i, int& prow, int& col, int& gs) __attribute__((always_inline)) {
        const int w = 4 * i + wave;
        if (w < REG) {
            prow = w / BPR, col = 16 * (w % BPR) + (lane >> 2), gs = lane & 3;
        } else {
            int t = (w - REG) * 64 + lane;
            t = t < LEFTN ? t : LEFTN - 1;
            prow = t >> 3, col = 16 * PX + ((t & 7) >> 2), gs = t & 3;
        }
    };
    // the chunk whose patch is being loaded, as uniform values set once per step: the chunk's
    // first channel in image l_n, the byte strides of a row and a pixel, and the shift of the
    // coordinates (1 for the channels below Cl, read at half resolution). The tensors' bases and
    // strides are copied into registers once (opaque to the compiler, which would otherwise
    // reload them from the kernel arguments at every block and wait for the scalar loads).
    using gchar = const __attribute__((address_space(1))) char;  // global memory
    const char* xb0 = reinterpret_cast<const char*>(a.x + a.xo);
    const char* xlb0 = reinterpret_cast<const char*>(a.xl + a.xlo);
    int xs2 = 2 * a.xs, xls2 = 2 * a.xls;
    asm volatile("" : "+s"(xb0), "+s"(xlb0), "+s"(xs2), "+s"(xls2));
    gchar* xb = (gchar*)xb0;
    gchar* xlb = (gchar*)xlb0;
    gchar* c_base = xb;
    int c_rs = 0, c_ps = 0, c_sh = 0;
    auto plan_chunk = [&](int kc) __attribute__((always_inline)) {
        if (kc < Cl) {
            c_ps = xls2, c_rs = Wl * xls2, c_sh = 1;
            c_base = xlb + 2 * kc + (long long)l_n * Hl * c_rs;
        } else {
            c_ps = xs2, c_rs = W * xs2, c_sh = 0;
            c_base = xb + 2 * (kc - Cl) + (long long)l_n * H * c_rs;
        }
    };
    // load block i of the planned chunk into the staging registers: a uniform base and a 32-bit
    // per-lane byte offset (24-bit products: rows of at most 16 MB, checked on the host). A row
    // segment takes its row in the base (scalar arithmetic, the circular wrap included) and the
    // lane's column offset c_xoff, computed once per step; other blocks compute both per lane.
    short8_t stage[NBW];
    unsigned c_xoff = 0;
    int c_y0 = 0;  // the patch row of this wave's first row segment, as an image row (unwrapped)
    auto plan_cols = [&]() __attribute__((always_inline)) {
        const int xx = wrap_near(l_tx0 + r_col - 1, W);
        c_xoff = __umul24((unsigned)(xx >> c_sh), (unsigned)c_ps) + 16 * r_gg;
        c_y0 = l_ty0 - 1 + wave / BPR;
    };
    auto issue_block = [&](int i) __attribute__((always_inline)) {
        using gs8 = const __attribute__((address_space(1))) short8_t;
        if (all_rows(i)) {
            // row segments of wave w: patch rows w / BPR + i (4 / BPR)
            // (only the first can lie above the image)
            const int y = c_y0 + i * (4 / BPR), yy = i == 0 ? wrap_near(y, H) : (y >= H ? y - H : y);
            stage[i] = *reinterpret_cast<gs8*>(c_base + (unsigned)((yy >> c_sh) * c_rs) + c_xoff);
        } else {
            int prow, col, gs;
            piece(i, prow, col, gs);
            const int yy = wrap_near(l_ty0 + prow - 1, H), xx = wrap_near(l_tx0 + col - 1, W);
            const unsigned off = __umul24((unsigned)(yy >> c_sh), (unsigned)c_rs) +
                                 __umul24((unsigned)(xx >> c_sh), (unsigned)c_ps) + 16 * (gs ^ ((col >> 1) & 3));
            stage[i] = *reinterpret_cast<gs8*>(c_base + off);
        }
    };
    // the staged pieces into LDS buffer buf
    auto publish = [&](int buf) __attribute__((always_inline)) {
        uint8_t* b = wconv_lds + buf * G::BUF_BYTES;
#pragma unroll
        for (int i = 0; i < NBW; ++i) {
            if (all_rows(i)) {
                const int w = 4 * i + wave;
                *reinterpret_cast<short8_t*>(b + (w / BPR) * PCOL * 64 + rb * 1024 + lane * 16) = stage[i];
            } else {
                int prow, col, gs;
                piece(i, prow, col, gs);
                *reinterpret_cast<short8_t*>(b + (prow * PCOL + col) * 64 + gs * 16) = stage[i];
            }
        }
    };
    // A operands of the three taps (0, dx), (1, dx), (2, dx): lane jl + 16 q holds
    // w[co][tap][kc + 8q .. +7] of channel co = base + 8 (jl / 4) + 4 jj + jl % 4 (a uniform base
    // and one per-lane byte offset). Row i of the product for half jj is then channel
    // 8 (i / 4) + 4 jj + i % 4, so that lane j + 16 g ends with channels 8g .. 8g+7 of pixel j
    // (elements 0..3 of half 0, then of half 1): 16 contiguous bytes of bf16 output.
    const unsigned woff = (unsigned)(((8 * (jl >> 2) + (jl & 3)) * 9 * Cin + 8 * q) * 2);
    auto load_w = [&](int it, int kc, int dx, short8_t (&wr)[9][2]) __attribute__((always_inline)) {
        const bf16* wb = a.w + ((it % groups) * 32 * CG + 32 * cg) * 9 * Cin + kc;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
                wr[3 * dy + dx][jj] = *reinterpret_cast<const short8_t*>(
                    reinterpret_cast<const char*>(wb + (4 * jj * 9 + 3 * dy + dx) * Cin) + woff);
    };
    // B operands: lane jl + 16 q reads pixel column 16 pxb + jl + dx of a patch row, channels
    // 8q .. 8q+7 of the chunk
    int boff[3];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
        const int col = 16 * pxb + jl + dx;
        boff[dx] = col * 64 + 16 * (q ^ ((col >> 1) & 3));
    }

    float4_t acc[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = float4_t{0.f, 0.f, 0.f, 0.f};

    // ---- epilogue of a finished item, one output row at a time -------------------------------
    int e_n = 0, e_ty0 = 0, e_xx = 0, e_cb = 0;
    bool e_xin = false;
    float e_bias[2][4];
    auto begin_item_out = [&](int it) __attribute__((always_inline)) {
        const int cgp = it % groups;
        int t = it / groups;
        const int tx = t % tiles_x;
        t /= tiles_x;
        e_ty0 = (t % tiles_y) * R;
        e_n = t / tiles_y;
        e_xx = tx * 16 * PX + 16 * pxb + jl;
        e_cb = cgp * 32 * CG + 32 * cg;
        e_xin = e_xx < W;
    };
    // the bias of the item's channels, from its copy in LDS
    auto load_bias = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const float4 b = *reinterpret_cast<const float4*>(s_bias + e_cb + 8 * q + 4 * jj);
            e_bias[jj][0] = b.x, e_bias[jj][1] = b.y, e_bias[jj][2] = b.z, e_bias[jj][3] = b.w;
        }
    };
    // the fused head's A operand: lane c + 16 g holds hw[c][8g .. 8g+7], the channels of the
    // bf16 outputs in lane g's B operand; and the head's bias. With 4 outputs the 4 weight rows
    // are repeated in A's rows 4..15, so that every lane group of the product holds the pixel's
    // 4 outputs (lane j + 16 g, element c: D[4g + c][j] = out c).
    short8_t head_a = {0, 0, 0, 0, 0, 0, 0, 0};
    float head_b[4] = {0.f, 0.f, 0.f, 0.f};
    if (CG == 1 && (OUT == kOutHead || (OUT == kOutAny && a.hw))) {
        const bool rep = OUT == kOutHead || a.rc == 4;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int ch = 8 * q + e;
            if (rep) head_a[e] = (short)a.hw[(jl & 3) * Cout + ch];
            else if (jl < a.rc) head_a[e] = (short)a.hw[jl * Cout + ch];
        }
        // with 4 outputs every lane adds them (rows are spread over the lanes, below)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = (OUT == kOutHead || a.rc == 4) ? e : 4 * q + e;
            if (a.hb && c < a.rc) head_b[e] = a.hb[c];
        }
    }
    uint32_t prev_bf[2][2];  // bf16 outputs of the previous (even) row, for the pool
    auto epi_row = [&](int r, const float4& res_row) __attribute__((always_inline)) {
        const int yy = e_ty0 + r;
        const bool in = yy < H && e_xin;
        const int pix = (e_n * H + yy) * W + e_xx;
        float v[2][4];
        uint32_t vb[2][2];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float x = acc[r][jj][e] + e_bias[jj][e];
                if (RELU) x = fmaxf(x, 0.0f);
                v[jj][e] = x;
            }
            vb[jj][0] = pack_bf2(v[jj][0], v[jj][1]);
            vb[jj][1] = pack_bf2(v[jj][2], v[jj][3]);
        }
        // the lane's channels: c8 .. c8+3 (half 0) and c8+4 .. c8+7 (half 1)
        const int c8 = e_cb + 8 * q;
        if (OUT != kOutHead && in) {
            if (OUT != kOutAny || a.y)
                *reinterpret_cast<uint4*>(a.y + pix * a.ys + a.yo + c8) = make_uint4(vb[0][0], vb[0][1], vb[1][0], vb[1][1]);
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                const int c4 = c8 + 4 * jj;
                if (OUT == kOutAny && a.yf)
                    *reinterpret_cast<float4*>(a.yf + pix * Cout + c4) = make_float4(v[jj][0], v[jj][1], v[jj][2], v[jj][3]);
                if (OUT == kOutAny && a.pred && !a.hw) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (c4 + e < a.rc) a.pred[pix * a.rc + c4 + e] = a.res[pix * a.rc + c4 + e] + v[jj][e];
                }
            }
        }
        if (OUT == kOutYPool || (OUT == kOutAny && a.yp)) {
            if (r & 1) {
                // 2x2 mean of the bf16 outputs: rows r-1, r are this lane's, the odd column is
                // the neighbouring lane's; summed in the order (0,0), (0,1), (1,0), (1,1)
                const int Hp = H >> 1, Wp = W >> 1, Y = (e_ty0 + r) >> 1, X = e_xx >> 1;
                uint32_t pb[2][2];
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                    float sm[4];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const float a0 = bf_lo(prev_bf[jj][h2]), a1 = bf_lo(vb[jj][h2]);
                        const float b0 = bf_hi(prev_bf[jj][h2]), b1 = bf_hi(vb[jj][h2]);
                        sm[2 * h2] = ((a0 + swap_lane_pair(a0)) + a1) + swap_lane_pair(a1);
                        sm[2 * h2 + 1] = ((b0 + swap_lane_pair(b0)) + b1) + swap_lane_pair(b1);
                    }
                    pb[jj][0] = pack_bf2(0.25f * sm[0], 0.25f * sm[1]);
                    pb[jj][1] = pack_bf2(0.25f * sm[2], 0.25f * sm[3]);
                }
                if ((jl & 1) == 0 && Y < Hp && X < Wp)
                    *reinterpret_cast<uint4*>(a.yp + ((e_n * Hp + Y) * Wp + X) * a.yps + a.ypo + c8) =
                        make_uint4(pb[0][0], pb[0][1], pb[1][0], pb[1][1]);
            } else {
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) prev_bf[jj][0] = vb[jj][0], prev_bf[jj][1] = vb[jj][1];
            }
        }
        if (CG == 1 && (OUT == kOutHead || (OUT == kOutAny && a.hw))) {
            // head output c of pixel jl lands in lane jl + 16 (c / 4), element c % 4, and with
            // 4 outputs in every lane jl + 16 g (the operand order: see head_a)
            short8_t hb;
            hb[0] = (short)(vb[0][0] & 0xffff); hb[1] = (short)(vb[0][0] >> 16);
            hb[2] = (short)(vb[0][1] & 0xffff); hb[3] = (short)(vb[0][1] >> 16);
            hb[4] = (short)(vb[1][0] & 0xffff); hb[5] = (short)(vb[1][0] >> 16);
            hb[6] = (short)(vb[1][1] & 0xffff); hb[7] = (short)(vb[1][1] >> 16);
            const float4_t d = mfma32(head_a, hb, float4_t{0.f, 0.f, 0.f, 0.f});
            if (OUT == kOutHead || a.rc == 4) {
                // every lane holds its pixel's 4 outputs; lane jl + 16 (r % 4) holds the
                // residual of this row and writes the prediction
                if (q == (r & 3) && in) {
                    const float4 rs = res_row;
                    *reinterpret_cast<float4*>(a.pred + pix * 4) =
                        make_float4(rs.x + (d[0] + head_b[0]), rs.y + (d[1] + head_b[1]),
                                    rs.z + (d[2] + head_b[2]), rs.w + (d[3] + head_b[3]));
                }
            } else if (OUT == kOutAny && in) {
                {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = 4 * q + e;
                        if (c < a.rc) a.pred[pix * a.rc + c] = a.res[pix * a.rc + c] + (d[e] + head_b[e]);
                    }
                }
            }
        }
    };

    // the item's output rows. With the fused head and 4 fields, lane jl + 16 k first reads the
    // residual of rows k, k+4, k+8, k+12 of pixel jl (rows outside the image read a clamped
    // one), so that every load is issued before the first store
    auto epilogue = [&]() __attribute__((always_inline)) {
        constexpr bool HEAD = CG == 1 && (OUT == kOutHead || OUT == kOutAny);
        float4 rq[R / 4];
#pragma unroll
        for (int m = 0; m < R / 4; ++m) rq[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (HEAD && a.hw && (OUT == kOutHead || a.rc == 4)) {
            const int xc = e_xx < W ? e_xx : W - 1;
#pragma unroll
            for (int m = 0; m < R / 4; ++m) {
                const int yr = e_ty0 + 4 * m + q, yy = yr < H ? yr : H - 1;
                rq[m] = *reinterpret_cast<const float4*>(a.res + ((e_n * H + yy) * W + xc) * 4);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) epi_row(r, rq[r / 4]);
    };
    // ---- the MFMAs of one step -----------------------------------------------------------------
    // by horizontal tap dx and patch row, with the next step's patch loads between the first
    // column's rows; once a tap column is done its registers take the next step's weights
    // (next_it, next_kc). B fragment t (column t / (R+2), patch row t % (R+2)) is read D
    // fragments ahead of its MFMAs, across column ends: 3 (about 12-18 MFMAs, more than the
    // LDS latency) where the 32-channel item's registers leave room for the extra fragments,
    // else 1 (with more, the compiler moves the reads back next to their MFMAs).
    short8_t wr[9][2];
    auto compute = [&](int buf, int next_it, int next_kc) __attribute__((always_inline)) {
        const uint8_t* base = wconv_lds + buf * G::BUF_BYTES;
        constexpr int T = 3 * (R + 2), D = CG == 1 ? 3 : 1;
        auto frag = [&](int t) __attribute__((always_inline)) {
            return *reinterpret_cast<const short8_t*>(base + (t % (R + 2)) * PCOL * 64 + boff[t / (R + 2)]);
        };
        short8_t bq[D + 1];
#pragma unroll
        for (int t = 0; t < D; ++t) bq[t] = frag(t);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
            for (int ir = 0; ir < R + 2; ++ir) {
                const int t = dx * (R + 2) + ir;
                if (t + D < T) bq[(t + D) % (D + 1)] = frag(t + D);
                const short8_t bx = bq[t % (D + 1)];
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int orow = ir - dy;
                    if (orow < 0 || orow >= R) continue;
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj) acc[orow][jj] = mfma32(wr[3 * dy + dx][jj], bx, acc[orow][jj]);
                }
                if (dx == 0) {
                    // this column's 18 rows carry up to 18 load blocks, the rest go after it
                    if (ir < NBW) issue_block(ir);
                    if (ir == R + 1)
#pragma unroll
                        for (int i = R + 2; i < NBW; ++i) issue_block(i);
                }
            }
            // compiler barriers keep the weight loads here, ahead of the next step, to which the
            // compiler would otherwise move them and wait for them at once; the last column's
            // go after the epilogue (below)
            if (dx < 2) {
                asm volatile("" ::: "memory");
                load_w(next_it, next_kc, dx, wr);
                asm volatile("" ::: "memory");
            }
        }
    };

    for (int c = tid; c < Cout; c += 256) s_bias[c] = a.bias ? a.bias[c] : 0.0f;
    int kc = 0, buf = 0;
    plan_loads(item);
    plan_chunk(0);
    plan_cols();
#pragma unroll
    for (int i = 0; i < NBW; ++i) issue_block(i);
    // the patch before the weights (the first step's top then waits for the patch only)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) load_w(item, 0, dx, wr);
    asm volatile("" ::: "memory");
    for (;;) {
        int nitem = item, nkc = kc + 32;
        if (nkc >= Cin) {
            nkc = 0;
            nitem = item + nloc;
        }
        const bool more = nitem < band1;
        // the loads for the next step are issued on every path, so that the compiler counts
        // outstanding loads exactly (it counts only loads every path issues); after the last
        // step they fetch this step's data again, which nothing reads
        const int lit = more ? nitem : item, lkc = more ? nkc : kc;
        // this step's patch goes from the staging registers into buffer buf, which every wave
        // finished reading two steps ago (the barrier of the last step is behind that); after
        // the barrier every wave's pieces are there. Fence-free barrier (__syncthreads' release
        // would wait for every outstanding load); compiler barriers keep memory accesses on
        // their side.
        publish(buf);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the stores above (and the bias)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (more && nkc == 0) plan_loads(nitem);
        plan_chunk(lkc);
        plan_cols();
        compute(buf, lit, lkc);
        if (nkc == 0) {
            begin_item_out(item);
            load_bias();
            epilogue();
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = float4_t{0.f, 0.f, 0.f, 0.f};
        }
        // the step's loads (and an item's stores) complete before more loads are issued: with
        // stores and loads outstanding together the compiler can no longer count loads in order
        // and waits for all of them wherever it needs one; and with the same loads outstanding
        // on both paths (item finished or not) it counts exactly at the next step's top, where
        // nothing then waits for the next step's patch
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
        asm volatile("" ::: "memory");
        load_w(lit, lkc, 2, wr);
        asm volatile("" ::: "memory");
        if (!more) break;
        item = nitem;
        kc = nkc;
        buf ^= 1;
    }
}

// dgrad weights: W'[ci][tap'][co] = W[co][KS*KS-1-tap'][ci], so that the data gradient of a
// circular convolution is the forward convolution of the output gradient with W'
__global__ void flip_weights_kernel(const bf16* __restrict__ w, bf16* __restrict__ wt, int Cout,
                                    int Cin, int taps) {
    const long long n = (long long)Cout * taps * Cin;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(i % Cin);
        const int tap = (int)((i / Cin) % taps);
        const int co = (int)(i / ((long long)Cin * taps));
        wt[((long long)ci * taps + (taps - 1 - tap)) * Cout + co] = w[i];
    }
}

// Weight gradient partials: part[chunk][co][tap][ci] = sum over the chunk's pixels p of
// dy[p, co] x[p + off(tap), ci]; bias partial bpart[chunk][co] = sum_p dy[p, co].
// An implicit GEMM with the pixels as the contraction: M = output channels, N = input
// channels, K = pixels, on the 16x16x32 MFMA. A workgroup of 4 waves owns COT output channels
// x 64 input channels (wave w: channels 16w .. 16w+15) and walks the 8 x 16 pixel tiles of
// its chunk; per tile the output gradient and the input patch (with its KS-1 halo, circular)
// are staged in LDS in their NHWC order, and every fragment (8 consecutive pixels of one
// channel per lane) is gathered with 2-byte LDS reads. Rows are padded to 68 bf16 so that the
// four 8-pixel groups of a fragment fall on different banks. All KS*KS taps accumulate at
// once; the bias is one more MFMA against a fragment of ones. Pixels beyond a ragged image
// edge carry a zero output gradient.
constexpr int kWgTH = 8, kWgTW = 16, kWgCIT = 64;

template <int KS, int COT>
__global__ __launch_bounds__(256) void wgrad_tile_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                                         int Cout, const bf16* __restrict__ x, int xs,
                                                         int xo, int Cin, int N, int H, int W,
                                                         int tiles_per_chunk, float* __restrict__ part,
                                                         float* __restrict__ bpart) {
    constexpr int TH = kWgTH, TW = kWgTW, NPX = TH * TW, CIT = kWgCIT;
    constexpr int HALO = KS - 1, XH = TH + HALO, XW = TW + HALO, T = KS * KS;
    constexpr int DYP = COT + 4, XP = CIT + 4, NF = COT / 16;
    __shared__ __attribute__((aligned(16))) bf16 s_dy[NPX * DYP];
    __shared__ __attribute__((aligned(16))) bf16 s_x[XH * XW * XP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int co0 = blockIdx.x * COT, ci0 = blockIdx.y * CIT, chunk = blockIdx.z;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = N * tiles_x * tiles_y;
    const int t_begin = chunk * tiles_per_chunk;
    const int t_end = min(ntiles, t_begin + tiles_per_chunk);
    const int h0 = HALO / 2;
    const bool bias_wave = blockIdx.y == 0 && wave == 0;
    const int g = lane >> 4, i = lane & 15;

    float4_t acc[NF][T], accb[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        accb[f] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < T; ++t) acc[f][t] = {0.f, 0.f, 0.f, 0.f};
    }
    short8_t ones;
#pragma unroll
    for (int k = 0; k < 8; ++k) ones[k] = (short)0x3f80;  // bf16 1.0

    for (int t = t_begin; t < t_end; ++t) {
        const int tx0 = (t % tiles_x) * TW, ty0 = ((t / tiles_x) % tiles_y) * TH;
        const int n = t / (tiles_x * tiles_y);
        __syncthreads();  // the previous tile's fragments have been read
        for (int piece = tid; piece < NPX * (COT / 8); piece += 256) {
            const int q = piece % (COT / 8), pix = piece / (COT / 8);
            const int yy = ty0 + pix / TW, xx = tx0 + pix % TW, co = co0 + 8 * q;
            short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (yy < H && xx < W && co < Cout)
                v = *reinterpret_cast<const short8_t*>(dy + ((size_t)(n * H + yy) * W + xx) * dys + dyo + co);
            short4_t* d = reinterpret_cast<short4_t*>(s_dy + pix * DYP + 8 * q);
            d[0] = short4_t{v[0], v[1], v[2], v[3]};
            d[1] = short4_t{v[4], v[5], v[6], v[7]};
        }
        for (int piece = tid; piece < XH * XW * (CIT / 8); piece += 256) {
            const int q = piece % (CIT / 8), pix = piece / (CIT / 8);
            const int sy = wrap_coord(ty0 + pix / XW - h0, H), sx = wrap_coord(tx0 + pix % XW - h0, W);
            const int ci = ci0 + 8 * q;
            short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (ci < Cin)
                v = *reinterpret_cast<const short8_t*>(x + ((size_t)(n * H + sy) * W + sx) * xs + xo + ci);
            short4_t* d = reinterpret_cast<short4_t*>(s_x + pix * XP + 8 * q);
            d[0] = short4_t{v[0], v[1], v[2], v[3]};
            d[1] = short4_t{v[4], v[5], v[6], v[7]};
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < NPX / 32; ++ks) {
            // this lane's 8 pixels of the 32-pixel K step: row 2 ks + g/2, columns 8 (g&1) + 0..7
            const int prow = 2 * ks + (g >> 1), pcol = 8 * (g & 1);
            short8_t af[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int e = 0; e < 8; ++e) af[f][e] = (short)s_dy[(prow * TW + pcol + e) * DYP + 16 * f + i];
#pragma unroll
            for (int tap = 0; tap < T; ++tap) {
                const int ddy = KS == 3 ? tap / 3 - 1 : 0, ddx = KS == 3 ? tap % 3 - 1 : 0;
                short8_t bf;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    bf[e] = (short)s_x[((prow + ddy + h0) * XW + pcol + e + ddx + h0) * XP + 16 * wave + i];
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f][tap] = mfma32(af[f], bf, acc[f][tap]);
            }
            if (bias_wave) {
#pragma unroll
                for (int f = 0; f < NF; ++f) accb[f] = mfma32(af[f], ones, accb[f]);
            }
        }
    }
    // D: lane (i + 16 g) holds rows 4g .. 4g+3 (output channels) of column i (input channel)
    const int ci = ci0 + 16 * wave + i;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = co0 + 16 * f + 4 * g + e;
            if (co >= Cout) continue;
            if (ci < Cin) {
#pragma unroll
                for (int tap = 0; tap < T; ++tap)
                    part[(((size_t)chunk * Cout + co) * T + tap) * Cin + ci] = acc[f][tap][e];
            }
            if (bias_wave && i == 0) bpart[(size_t)chunk * Cout + co] = accb[f][e];
        }
}

// Deterministic sum over chunks: out[i] = sum_c part[c][i]. A workgroup takes 16 consecutive
// indices; its 16 chunk lanes each sum the chunks c = lane, lane + 16, ... in order, and the
// 16 lane sums are added in lane order.
__global__ __launch_bounds__(256) void sum_chunks_kernel(const float* __restrict__ part, long long n,
                                                         int nchunks, float* __restrict__ out) {
    __shared__ float sh[16][17];
    const int j = threadIdx.x & 15, cl = threadIdx.x >> 4;
    for (long long i0 = (long long)blockIdx.x * 16; i0 < n; i0 += (long long)gridDim.x * 16) {
        const long long i = i0 + j;
        float s = 0.0f;
        if (i < n)
            for (int c = cl; c < nchunks; c += 16) s += part[(long long)c * n + i];
        sh[cl][j] = s;
        __syncthreads();
        if (cl == 0 && i < n) {
            float t = 0.0f;
            for (int k = 0; k < 16; ++k) t += sh[k][j];
            out[i] = t;
        }
        __syncthreads();
    }
}

// Elementwise kernels on NHWC bf16 slices, 8 channels (one 16-byte piece) per thread: block b
// walks image rows b, b + gridDim.x, ... (row = n * rows_per_image + y); the threads of a block
// walk the (pixel, piece) pairs of the row. C, channel strides and offsets are multiples of 8.
__device__ __forceinline__ short8_t ld8(const bf16* p) { return *reinterpret_cast<const short8_t*>(p); }
__device__ __forceinline__ void st8(bf16* p, short8_t v) { *reinterpret_cast<short8_t*>(p) = v; }
__device__ __forceinline__ float s2f(short s) { return bf2f((bf16)s); }

// 2x2 average pool: y[n, Y, X, c] = mean of x[n, 2Y..2Y+1, 2X..2X+1, c] (H x W input)
__global__ __launch_bounds__(256) void avgpool_kernel(const bf16* __restrict__ x, int xs, int xo,
                                                      bf16* __restrict__ y, int ys, int yo, int C,
                                                      int N, int H, int W) {
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    for (int row = blockIdx.x; row < N * Ho; row += gridDim.x) {
        const int nn = row / Ho, Y = row % Ho;
        const size_t b0 = (size_t)(nn * H + 2 * Y) * W;
        for (int j = threadIdx.x; j < Wo * C8; j += blockDim.x) {
            const int X = j / C8, c = 8 * (j % C8);
            const size_t b = b0 + 2 * X;
            const short8_t v0 = ld8(x + b * xs + xo + c), v1 = ld8(x + (b + 1) * xs + xo + c);
            const short8_t v2 = ld8(x + (b + W) * xs + xo + c), v3 = ld8(x + (b + W + 1) * xs + xo + c);
            short8_t o;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                o[k] = (short)f2bf(0.25f * (s2f(v0[k]) + s2f(v1[k]) + s2f(v2[k]) + s2f(v3[k])));
            st8(y + ((size_t)row * Wo + X) * ys + yo + c, o);
        }
    }
}

// gradient of the pool added into the input-gradient slice: dx[p] += dy[parent(p)] / 4
__global__ __launch_bounds__(256) void avgpool_bwd_add_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                                              bf16* __restrict__ dx, int dxs, int dxo,
                                                              int C, int N, int H, int W) {
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    for (int row = blockIdx.x; row < N * H; row += gridDim.x) {
        const int nn = row / H, yy = row % H;
        const size_t q0 = (size_t)(nn * Ho + yy / 2) * Wo;
        for (int j = threadIdx.x; j < W * C8; j += blockDim.x) {
            const int xx = j / C8, c = 8 * (j % C8);
            bf16* d = dx + ((size_t)row * W + xx) * dxs + dxo + c;
            const short8_t g = ld8(dy + (q0 + xx / 2) * dys + dyo + c), v = ld8(d);
            short8_t o;
#pragma unroll
            for (int k = 0; k < 8; ++k) o[k] = (short)f2bf(s2f(v[k]) + 0.25f * s2f(g[k]));
            st8(d, o);
        }
    }
}

// nearest 2x upsample: y[n, y, x, c] = x[n, y/2, x/2, c] (output H x W)
__global__ __launch_bounds__(256) void upsample_kernel(const bf16* __restrict__ x, int xs, int xo,
                                                       bf16* __restrict__ y, int ys, int yo, int C,
                                                       int N, int H, int W) {
    const int Hi = H / 2, Wi = W / 2, C8 = C / 8;
    for (int row = blockIdx.x; row < N * H; row += gridDim.x) {
        const int nn = row / H, yy = row % H;
        const size_t q0 = (size_t)(nn * Hi + yy / 2) * Wi;
        for (int j = threadIdx.x; j < W * C8; j += blockDim.x) {
            const int xx = j / C8, c = 8 * (j % C8);
            st8(y + ((size_t)row * W + xx) * ys + yo + c, ld8(x + (q0 + xx / 2) * xs + xo + c));
        }
    }
}

// gradient of the upsample: dx[q, c] = sum of dy over the 4 children of q (dy is H x W)
__global__ __launch_bounds__(256) void upsample_bwd_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                                           bf16* __restrict__ dx, int dxs, int dxo,
                                                           int C, int N, int H, int W) {
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    for (int row = blockIdx.x; row < N * Ho; row += gridDim.x) {
        const int nn = row / Ho, Y = row % Ho;
        const size_t b0 = (size_t)(nn * H + 2 * Y) * W;
        for (int j = threadIdx.x; j < Wo * C8; j += blockDim.x) {
            const int X = j / C8, c = 8 * (j % C8);
            const size_t b = b0 + 2 * X;
            const short8_t v0 = ld8(dy + b * dys + dyo + c), v1 = ld8(dy + (b + 1) * dys + dyo + c);
            const short8_t v2 = ld8(dy + (b + W) * dys + dyo + c), v3 = ld8(dy + (b + W + 1) * dys + dyo + c);
            short8_t o;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                o[k] = (short)f2bf(s2f(v0[k]) + s2f(v1[k]) + s2f(v2[k]) + s2f(v3[k]));
            st8(dx + ((size_t)row * Wo + X) * dxs + dxo + c, o);
        }
    }
}

// ReLU gradient in place: g *= (a > 0), a the post-activation of the same slice layout;
// npix pixels taken as rows of 64 pixels (the last one partial)
__global__ __launch_bounds__(256) void relu_bwd_kernel(bf16* __restrict__ g, int gs, int go,
                                                       const bf16* __restrict__ a, int as, int ao,
                                                       int C, long long npix) {
    const int C8 = C / 8;
    const long long rows = (npix + 63) / 64;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const long long p0 = row * 64;
        const int w = (int)min(64LL, npix - p0);
        for (int j = threadIdx.x; j < w * C8; j += blockDim.x) {
            const size_t p = (size_t)(p0 + j / C8);
            const int c = 8 * (j % C8);
            const short8_t av = ld8(a + p * as + ao + c);
            short8_t gv = ld8(g + p * gs + go + c);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (!(s2f(av[k]) > 0.0f)) gv[k] = 0;
            st8(g + p * gs + go + c, gv);
        }
    }
}

// pack network input: x0 (bf16, 16 channels, zero beyond cin) from FP32 NHWC [.., cin]
__global__ __launch_bounds__(256) void pack_input_kernel(const float* __restrict__ in, int cin,
                                                         bf16* __restrict__ x0, long long npix) {
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < npix; p += (long long)gridDim.x * 256) {
        short8_t lo = {0, 0, 0, 0, 0, 0, 0, 0}, hi = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c >= cin) break;
            const short v = (short)f2bf(in[p * cin + c]);
            if (c < 8) lo[c] = v; else hi[c - 8] = v;
        }
        st8(x0 + p * 16, lo);
        st8(x0 + p * 16 + 8, hi);
    }
}

// prediction = input + head residual (first cout channels of the FP32 head output);
// with a target: squared-error partials per workgroup and dY = 2 w_c (pred - target) / count
// as bf16 into the 16-channel head-gradient buffer
__global__ __launch_bounds__(256) void predict_loss_kernel(const float* __restrict__ in,
                                                           const float* __restrict__ head, int cout,
                                                           float* __restrict__ pred,
                                                           const float* __restrict__ target,
                                                           const float* __restrict__ wch,
                                                           bf16* __restrict__ dy, long long npix,
                                                           float inv_count,
                                                           double* __restrict__ part) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < npix; p += (long long)gridDim.x * 256) {
        for (int c = 0; c < 16; ++c) {
            if (c < cout) {
                const float v = in[p * cout + c] + head[p * 16 + c];
                if (pred) pred[p * cout + c] = v;
                if (target) {
                    const float d = v - target[p * cout + c];
                    const float wc = wch ? wch[c] : 1.0f;
                    acc += (double)(wc * d * d);
                    dy[p * 16 + c] = f2bf(2.0f * wc * d * inv_count);
                }
            } else if (target) {
                dy[p * 16 + c] = 0;
            }
        }
    }
    if (!part) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Adam on FP32 master weights with bias-corrected moments, refreshing the bf16 copy
__global__ void adam_kernel(float* __restrict__ w, bf16* __restrict__ wb, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        w[i] = wi;
        wb[i] = f2bf(wi);
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ a, bf16* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = f2bf(a[i]);
}

__global__ void bf16_to_f32_kernel(const bf16* __restrict__ b, float* __restrict__ a, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = bf2f(b[i]);
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
static dim3 row_grid(long long rows) { return dim3((unsigned)(rows < 65536 ? (rows < 1 ? 1 : rows) : 65536)); }

static dim3 ew_grid(long long n) {
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t unet_mfma_probe(int k32, const bf16* A, const bf16* B, float* D, hipStream_t st) {
    if (k32)
        hipLaunchKernelGGL(mfma32_probe_kernel, dim3(1), dim3(64), 0, st, A, B, D);
    else
        hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, st, A, B, D);
    return hipGetLastError();
}

template <int KS, bool R, int C, bool PFW>
static hipError_t launch_conv_pf(const ConvArgs& a, dim3 grid, hipStream_t st) {
    constexpr size_t lds = (size_t)conv_lds_elems<KS, C>() * sizeof(bf16);
    static bool attr = false;  // dynamic LDS above 64 KiB must be requested once per kernel
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)&conv_tile_kernel<KS, R, C, PFW>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((conv_tile_kernel<KS, R, C, PFW>), grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

template <int KS, bool R, int C>
static hipError_t launch_conv_t(const ConvArgs& a, bool pfw, hipStream_t st) {
    const long long tiles = (long long)a.N * ((a.H + kConvTR - 1) / kConvTR) * ((a.W + kConvTC - 1) / kConvTC);
    dim3 grid((unsigned)tiles, (unsigned)((a.Cout + C - 1) / C));
    return pfw ? launch_conv_pf<KS, R, C, true>(a, grid, st) : launch_conv_pf<KS, R, C, false>(a, grid, st);
}

// LDS of the first layer: its patch and staged weights, or the epilogue's bf16 output tile (it has
// no fused head, so nothing beyond the tile), whichever is larger; 20 KB at C = 32, which leaves
// room for six workgroups per CU, as many as its registers allow
template <int C>
constexpr int conv_first_lds_elems() {
    constexpr int in = (kConvTR + 2) * (kConvTC + 2) * 4 + C * 9 * 4;
    constexpr int out = kConvTR * kConvTC * (C + 8);
    return in > out ? in : out;
}

template <bool R, int C>
static hipError_t launch_first_t(const ConvArgs& a, hipStream_t st) {
    if (a.hw) return hipErrorInvalidValue;  // the LDS below holds no head outputs
    constexpr size_t lds = (size_t)conv_first_lds_elems<C>() * sizeof(bf16);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)&conv_first_kernel<R, C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const long long tiles = (long long)a.N * ((a.H + kConvTR - 1) / kConvTR) * ((a.W + kConvTC - 1) / kConvTC);
    dim3 grid((unsigned)tiles, (unsigned)((a.Cout + C - 1) / C));
    hipLaunchKernelGGL((conv_first_kernel<R, C>), grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

template <bool R>
static hipError_t launch_first_loop(const ConvArgs& a, hipStream_t st) {
    static int grid_cap = 0;  // workgroups resident at once on this device (set once)
    if (!grid_cap) {
        int dev = 0, cus = 0, per = 0;
        hipError_t e;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)&conv_first_loop_kernel<R>, 256, 0)) !=
            hipSuccess)
            return e;
        grid_cap = (per < 1 ? 1 : per) * cus;
    }
    const long long tiles = (long long)a.N * (a.H / kConvTR) * (a.W / kConvTC);
    const long long grid = tiles < grid_cap ? tiles : grid_cap;
    hipLaunchKernelGGL((conv_first_loop_kernel<R>), dim3((unsigned)grid), dim3(256), 0, st, a, (int)tiles);
    return hipGetLastError();
}

template <int CG, bool R, int OUT, int RW>
static hipError_t launch_wave_o(const ConvArgs& a, hipStream_t st) {
    using G = WaveConvGeom<CG, RW>;
    static int grid_cap = 0;  // workgroups resident at once on this device (set once)
    if (!grid_cap) {
        hipError_t e = hipFuncSetAttribute((const void*)&conv3_wave_kernel<CG, R, OUT, RW>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, G::LDS_BYTES);
        if (e != hipSuccess) return e;
        int dev = 0, cus = 0, per = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)&conv3_wave_kernel<CG, R, OUT, RW>, 256,
                                                              G::LDS_BYTES)) != hipSuccess)
            return e;
        grid_cap = (per < 1 ? 1 : per) * cus;
    }
    const long long items = (long long)a.N * ((a.H + RW - 1) / RW) *
                            ((a.W + 16 * G::PX - 1) / (16 * G::PX)) * (a.Cout / (32 * CG));
    if (items > (1LL << 30)) return hipErrorInvalidValue;
    long long grid = items < grid_cap ? items : grid_cap;
    if (grid < 8) grid = 8;  // every XCD band has a workgroup
    hipLaunchKernelGGL((conv3_wave_kernel<CG, R, OUT, RW>), dim3((unsigned)grid), dim3(256), G::LDS_BYTES, st, a, (int)items);
    return hipGetLastError();
}

template <int CG, bool R, int RW = kWvRows>
static hipError_t launch_wave_t(const ConvArgs& a, hipStream_t st) {
    if constexpr (CG == 1)
        if (a.hw && a.rc == 4 && !a.y && !a.yp && !a.yf) return launch_wave_o<CG, R, kOutHead, RW>(a, st);
    if (!a.hw && !a.yf && !a.pred && a.y) {
        if (a.yp) return launch_wave_o<CG, R, kOutYPool, RW>(a, st);
        return launch_wave_o<CG, R, kOutY, RW>(a, st);
    }
    return launch_wave_o<CG, R, kOutAny, RW>(a, st);
}

// the wave-row kernel unless LBPF_CONV_WAVE=0 is set (read once)
static bool wave_conv_enabled() {
    static const bool on = [] {
        const char* v = getenv("LBPF_CONV_WAVE");
        return !(v && v[0] == '0');
    }();
    return on;
}

hipError_t unet_conv_plan(int ks, const ConvArgs& a, ConvPlan* plan) {
    ConvPlan p{};
    if (a.xin) {
        const bool ok = ks == 3 && a.xin_c >= 1 && a.xin_c <= 4 && a.Cl == 0 && !a.hw &&
                        (!a.y || (a.Cout % 8 == 0 && a.ys % 8 == 0 && a.yo % 8 == 0)) &&
                        (!a.yp || (a.Cout % 8 == 0 && a.yps % 8 == 0 && a.ypo % 8 == 0 &&
                                   a.H % 2 == 0 && a.W % 2 == 0)) &&
                        (!a.pred || a.res) && a.N >= 1 && a.H >= 1 && a.W >= 1;
        if (!ok) return hipErrorInvalidValue;
        auto al = [](const void* ptr, int b) { return (reinterpret_cast<uintptr_t>(ptr) & (b - 1)) == 0; };
        // the persistent kernel: 4 fields, 32 channels, y and/or its pool only, whole tiles
        const bool loop = a.xin_c == 4 && a.Cin % 4 == 0 && a.Cout == 32 && (a.y || a.yp) && !a.yf && !a.pred &&
                          a.H % kConvTR == 0 && a.W % kConvTC == 0 && al(a.xin, 16) && al(a.w, 8) &&
                          (!a.y || al(a.y, 16)) && (!a.yp || al(a.yp, 16)) &&
                          (long long)a.N * (a.H / kConvTR) * (a.W / kConvTC) < (1LL << 30);
        p.first = loop ? 3 : 1;
        p.cot = a.Cout <= 32 ? 32 : 64;
        p.pfw = 0;
        *plan = p;
        return hipSuccess;
    }
    const bool aligned = a.Cin % 8 == 0 && a.xs % 8 == 0 && a.xo % 8 == 0 &&
                         (a.Cl == 0 || (a.Cl % 8 == 0 && a.xls % 8 == 0 && a.xlo % 8 == 0 &&
                                        a.H % 2 == 0 && a.W % 2 == 0)) &&
                         (!a.y || (a.Cout % 8 == 0 && a.ys % 8 == 0 && a.yo % 8 == 0)) &&
                         (!a.yp || (a.Cout % 8 == 0 && a.yps % 8 == 0 && a.ypo % 8 == 0 &&
                                    a.H % 2 == 0 && a.W % 2 == 0)) &&
                         (!a.pred || (a.res && a.rc <= a.Cout)) &&
                         (!a.hw || (a.pred && a.res && a.Cout <= 32 && a.rc >= 1 && a.rc <= 16));
    if (!aligned || (ks != 1 && ks != 3) || a.Cl > a.Cin || a.N < 1 || a.H < 1 || a.W < 1)
        return hipErrorInvalidValue;
    // 3x3 with whole 32-channel chunks and 32-channel output groups: the wave-row kernel
    auto al16 = [](const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; };
    const int wcot = a.Cout % 128 == 0 ? 128 : (a.Cout % 64 == 0 ? 64 : 32);
    if (ks == 3 && wave_conv_enabled() && a.Cin % 32 == 0 && a.Cl % 32 == 0 && a.Cout % 32 == 0 &&
        a.Cout <= kWaveMaxCout &&
        a.H >= kWvRows + 2 && a.W >= 16 * (128 / wcot) + 2 &&
        (long long)a.N * a.H * a.W * (a.Cin + a.Cout) < (1LL << 30) &&
        (long long)a.W * a.xs * 2 < (1LL << 24) && (a.Cl == 0 || (long long)(a.W >> 1) * a.xls * 2 < (1LL << 24)) &&
        (!a.hw || a.Cout == 32) && al16(a.x) && (a.Cl == 0 || al16(a.xl)) && al16(a.w) && (!a.yf || al16(a.yf)) &&
        (!a.y || al16(a.y)) && (!a.yp || al16(a.yp)) && (!a.hw || a.rc != 4 || (al16(a.res) && al16(a.pred)))) {
        p.first = 2;
        p.cot = wcot;
        // 128-channel work items of 8 rows instead of 16 when the 16-row ones would not give
        // every CU one (a 128^2 level: 128 items)
        const long long items16 = (long long)a.N * ((a.H + kWvRows - 1) / kWvRows) * ((a.W + 15) / 16) * (a.Cout / 128);
        p.pfw = (wcot == 128 && items16 < 256 && a.H >= kWvRowsHalf + 2) ? 1 : 0;
        *plan = p;
        return hipSuccess;
    }
    int cot = a.Cout <= 16 ? 16 : (a.Cout <= 32 ? 32 : 64);
    if (a.hw) cot = 32;  // the fused head needs every output channel in one workgroup
    // fewer than ~2 workgroups per CU with 64 channels each: take 32 (more workgroups)
    const long long tiles = (long long)a.N * ((a.H + kConvTR - 1) / kConvTR) * ((a.W + kConvTC - 1) / kConvTC);
    // a single input chunk gains nothing from the weight prefetch of COT = 64: take 32 at three
    // workgroups per CU when the grid fills them
    if (cot == 64 && a.Cin <= kConvCK && tiles * ((a.Cout + 31) / 32) >= 768) cot = 32;
    if (cot == 64 && tiles * ((a.Cout + 63) / 64) < 512) cot = 32;
    // COT = 32: three workgroups per CU without the weight prefetch pay off only when the grid
    // has enough workgroups to fill them (three per CU)
    p.first = 0;
    p.cot = cot;
    p.pfw = (cot >= 64 || tiles * ((a.Cout + cot - 1) / cot) < 768) ? 1 : 0;
    *plan = p;
    return hipSuccess;
}

hipError_t unet_conv(int ks, bool relu, const ConvArgs& a, hipStream_t st) {
    ConvPlan p;
    const hipError_t e = unet_conv_plan(ks, a, &p);
    if (e != hipSuccess) return e;
    if (p.first == 2) {
        if (p.cot == 128 && p.pfw)
            return relu ? launch_wave_t<4, true, kWvRowsHalf>(a, st) : launch_wave_t<4, false, kWvRowsHalf>(a, st);
        if (p.cot == 128) return relu ? launch_wave_t<4, true>(a, st) : launch_wave_t<4, false>(a, st);
        if (p.cot == 64) return relu ? launch_wave_t<2, true>(a, st) : launch_wave_t<2, false>(a, st);
        return relu ? launch_wave_t<1, true>(a, st) : launch_wave_t<1, false>(a, st);
    }
    if (p.first == 3) return relu ? launch_first_loop<true>(a, st) : launch_first_loop<false>(a, st);
    if (p.first) {
        if (p.cot == 32) return relu ? launch_first_t<true, 32>(a, st) : launch_first_t<false, 32>(a, st);
        return relu ? launch_first_t<true, 64>(a, st) : launch_first_t<false, 64>(a, st);
    }
    const bool pfw = p.pfw != 0;
#define LBPF_CONV(KS_, C_) return relu ? launch_conv_t<KS_, true, C_>(a, pfw, st) : launch_conv_t<KS_, false, C_>(a, pfw, st)
    if (ks == 3) {
        if (p.cot == 16) LBPF_CONV(3, 16);
        if (p.cot == 32) LBPF_CONV(3, 32);
        LBPF_CONV(3, 64);
    }
    if (p.cot == 16) LBPF_CONV(1, 16);
    if (p.cot == 32) LBPF_CONV(1, 32);
    LBPF_CONV(1, 64);
#undef LBPF_CONV
}

hipError_t unet_conv_fwd(int ks, bool relu, const bf16* x, int xs, int xo, int Cin, const bf16* w,
                         const float* bias, bf16* y, int ys, int yo, int Cout, float* yf, int N,
                         int H, int W, hipStream_t st) {
    ConvArgs a{};
    a.x = x; a.xs = xs; a.xo = xo;
    a.Cin = Cin; a.w = w; a.bias = bias;
    a.y = y; a.ys = ys; a.yo = yo; a.yf = yf;
    a.Cout = Cout; a.N = N; a.H = H; a.W = W;
    return unet_conv(ks, relu, a, st);
}

hipError_t unet_flip_weights(const bf16* w, bf16* wt, int Cout, int Cin, int taps, hipStream_t st) {
    hipLaunchKernelGGL(flip_weights_kernel, ew_grid((long long)Cout * Cin * taps), dim3(256), 0, st, w, wt, Cout, Cin, taps);
    return hipGetLastError();
}

hipError_t unet_conv_wgrad(int ks, const bf16* dy, int dys, int dyo, int Cout, const bf16* x, int xs,
                           int xo, int Cin, int N, int H, int W, int max_chunks, float* part,
                           float* bpart, float* dw, float* db, hipStream_t st) {
    if ((ks != 1 && ks != 3) || max_chunks < 1 || dys % 8 || dyo % 8 || xs % 8 || xo % 8 || Cout % 8 || Cin % 8)
        return hipErrorInvalidValue;
    const int taps = ks * ks;
    const long long ntiles = (long long)N * ((H + kWgTH - 1) / kWgTH) * ((W + kWgTW - 1) / kWgTW);
    const int cot = Cout <= 32 ? 32 : 64;
    const int gx = (Cout + cot - 1) / cot, gy = (Cin + kWgCIT - 1) / kWgCIT;
    // pixel chunks: about 1024 workgroups in all, within the partial buffer
    long long want = (1024 + gx * gy - 1) / (gx * gy);
    if (want > max_chunks) want = max_chunks;
    if (want > ntiles) want = ntiles;
    const int tpc = (int)((ntiles + want - 1) / want);
    const int chunks = (int)((ntiles + tpc - 1) / tpc);
    dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)chunks);
#define LBPF_WG(KS_, C_) hipLaunchKernelGGL((wgrad_tile_kernel<KS_, C_>), grid, dim3(256), 0, st, dy, dys, dyo, \
                                            Cout, x, xs, xo, Cin, N, H, W, tpc, part, bpart)
    if (ks == 3) { if (cot == 32) LBPF_WG(3, 32); else LBPF_WG(3, 64); }
    else { if (cot == 32) LBPF_WG(1, 32); else LBPF_WG(1, 64); }
#undef LBPF_WG
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nw = (long long)Cout * taps * Cin;
    hipLaunchKernelGGL(sum_chunks_kernel, row_grid((nw + 15) / 16), dim3(256), 0, st, part, nw, chunks, dw);
    hipLaunchKernelGGL(sum_chunks_kernel, row_grid((Cout + 15) / 16), dim3(256), 0, st, bpart, (long long)Cout, chunks, db);
    return hipGetLastError();
}

hipError_t unet_avgpool(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(avgpool_kernel, row_grid((long long)N * H / 2), dim3(256), 0, st, x, xs, xo, y, ys, yo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_avgpool_bwd_add(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(avgpool_bwd_add_kernel, row_grid((long long)N * H), dim3(256), 0, st, dy, dys, dyo, dx, dxs, dxo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_upsample(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(upsample_kernel, row_grid((long long)N * H), dim3(256), 0, st, x, xs, xo, y, ys, yo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_upsample_bwd(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(upsample_bwd_kernel, row_grid((long long)N * H / 2), dim3(256), 0, st, dy, dys, dyo, dx, dxs, dxo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_relu_bwd(bf16* g, int gs, int go, const bf16* a, int as, int ao, int C, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(relu_bwd_kernel, row_grid((npix + 63) / 64), dim3(256), 0, st, g, gs, go, a, as, ao, C, npix);
    return hipGetLastError();
}
hipError_t unet_pack_input(const float* in, int cin, bf16* x0, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(pack_input_kernel, ew_grid(npix), dim3(256), 0, st, in, cin, x0, npix);
    return hipGetLastError();
}
hipError_t unet_predict_loss(const float* in, const float* head, int cout, float* pred, const float* target,
                             const float* wch, bf16* dy, long long npix, double* part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(predict_loss_kernel, dim3(nblk), dim3(256), 0, st, in, head, cout, pred, target, wch, dy,
                       npix, 1.0f / (float)(npix * cout), part);
    return hipGetLastError();
}
hipError_t unet_adam(float* w, bf16* wb, const float* g, float* m, float* v, long long n, float lr, float b1,
                     float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, ew_grid(n), dim3(256), 0, st, w, wb, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}
hipError_t unet_to_bf16(const float* a, bf16* b, long long n, hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, ew_grid(n), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}
hipError_t unet_bf16_to_f32(const bf16* b, float* a, long long n, hipStream_t st) {
    hipLaunchKernelGGL(bf16_to_f32_kernel, ew_grid(n), dim3(256), 0, st, b, a, n);
    return hipGetLastError();
}

}  // namespace lbpf
