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

namespace lbpf {

typedef uint16_t bf16;
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

// Convolution with a KS x KS kernel (KS = 1 or 3), stride 1, circular padding:
//   y[p, co] = act( bias[co] + sum_{tap, ci} x[p + off(tap), ci] w[co, tap, ci] )
// as an implicit GEMM: M = pixels, N = output channels, K = KS*KS*Cin.
// x: NHWC bf16 with channel stride xs and offset xo (Cin channels used, Cin % 16 == 0)
// w: [Cout][KS*KS][Cin] bf16; bias: Cout floats (may be NULL)
// y: NHWC bf16 with channel stride ys and offset yo (Cout % 64 == 0 or the tail masked);
// yf: optional FP32 copy, NHWC with channel stride Cout.
// Workgroup: 4 waves; a wave computes 16 consecutive pixels x 64 output channels.
template <int KS, bool RELU>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const bf16* __restrict__ x, int xs, int xo,
                                                       int Cin, const bf16* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       bf16* __restrict__ y, int ys, int yo,
                                                       int Cout, float* __restrict__ yf, int N,
                                                       int H, int W) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long npix = (long long)N * H * W;
    const long long p0 = ((long long)blockIdx.x * 4 + wave) * 16;
    const int co0 = blockIdx.y * 64;
    if (p0 >= npix) return;
    // pixel of this lane's A row
    const long long pa = p0 + (lane & 15);
    const bool pa_ok = pa < npix;
    const long long pac = pa_ok ? pa : npix - 1;
    const int xa = (int)(pac % W), ya = (int)((pac / W) % H);
    const long long na = pac / ((long long)W * H);
    const int kq = 4 * (lane >> 4);  // first of this lane's four k within a 16-chunk
    float4_t acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = {0.f, 0.f, 0.f, 0.f};
    const int K = KS * KS * Cin;
    for (int tap = 0; tap < KS * KS; ++tap) {
        const int dy = KS == 3 ? tap / 3 - 1 : 0, dx = KS == 3 ? tap % 3 - 1 : 0;
        int sy = ya + dy, sx = xa + dx;
        sy = sy < 0 ? sy + H : (sy >= H ? sy - H : sy);
        sx = sx < 0 ? sx + W : (sx >= W ? sx - W : sx);
        const bf16* xp = x + ((na * H + sy) * W + sx) * xs + xo + kq;
        for (int kc = 0; kc < Cin; kc += 16) {
            const short4_t a = load4(xp + kc);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = co0 + 16 * j + (lane & 15);
                const short4_t b = co < Cout ? load4(w + (long long)co * K + tap * Cin + kc + kq)
                                             : short4_t{0, 0, 0, 0};
                acc[j] = mfma16(a, b, acc[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int co = co0 + 16 * j + (lane & 15);
        if (co >= Cout) continue;
        const float bb = bias ? bias[co] : 0.0f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long long p = p0 + 4 * (lane >> 4) + e;
            if (p >= npix) continue;
            float v = acc[j][e] + bb;
            if (RELU) v = fmaxf(v, 0.0f);
            y[p * ys + yo + co] = f2bf(v);
            if (yf) yf[p * Cout + co] = v;
        }
    }
}

// LDS-tiled convolution (same contract as conv_fwd_kernel): a workgroup of 4 waves computes a
// tile of 4 rows x 16 columns of one image (wave w: row w) for COT output channels. Per chunk
// of 32 input channels it stages the input patch (with its KS-1 halo, circular) and the
// weights of the COT channels in LDS, then every tap is one 16x16x32 MFMA per 16 output
// channels with the A fragment shared across them. The next chunk is loaded into registers
// while the current one is multiplied. Pixels beyond the image (a ragged tile) are computed
// from wrapped data and not stored.
template <int KS, bool RELU, int COT>
__global__ __launch_bounds__(256) void conv_lds_kernel(const bf16* __restrict__ x, int xs, int xo,
                                                       int Cin, const bf16* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       bf16* __restrict__ y, int ys, int yo,
                                                       int Cout, float* __restrict__ yf, int N,
                                                       int H, int W) {
    constexpr int TR = 4, TC = 16, CK = 32, CKP = 40;  // CKP: padded LDS row (bank spread)
    constexpr int HALO = KS - 1, PR = TR + HALO, PC = TC + HALO, T = KS * KS;
    constexpr int NPATCH = PR * PC * (CK / 8);           // 16-byte pieces of the patch
    constexpr int NWT = COT * T * (CK / 8);              // 16-byte pieces of the weights
    constexpr int PP = (NPATCH + 255) / 256, PW = (NWT + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 s_x[PR * PC * CKP];
    __shared__ __attribute__((aligned(16))) bf16 s_w[COT * T * CKP];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (W + TC - 1) / TC, tiles_y = (H + TR - 1) / TR;
    const int tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TC, ty0 = ((tile / tiles_x) % tiles_y) * TR;
    const long long n = tile / (tiles_x * tiles_y);
    const int co0 = blockIdx.y * COT;
    const int K = T * Cin;
    const int h0 = HALO / 2;

    short8_t rp[PP], rw[PW];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int piece = tid + 256 * i;
            short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (piece < NPATCH) {
                const int q = piece % (CK / 8), pix = piece / (CK / 8);
                const int pr = pix / PC, pc = pix % PC;
                int sy = ty0 + pr - h0, sx = tx0 + pc - h0;
                sy = ((sy % H) + H) % H;
                sx = ((sx % W) + W) % W;
                const int ci = kc + 8 * q;
                if (ci < Cin) v = *reinterpret_cast<const short8_t*>(x + ((n * H + sy) * W + sx) * xs + xo + ci);
            }
            rp[i] = v;
        }
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int piece = tid + 256 * i;
            short8_t v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (piece < NWT) {
                const int q = piece % (CK / 8), r = piece / (CK / 8);
                const int tap = r % T, col = r / T;
                const int co = co0 + col, ci = kc + 8 * q;
                if (co < Cout && ci < Cin) v = *reinterpret_cast<const short8_t*>(w + (long long)co * K + tap * Cin + ci);
            }
            rw[i] = v;
        }
    };
    auto publish = [&]() {
#pragma unroll
        for (int i = 0; i < PP; ++i) {
            const int piece = tid + 256 * i;
            if (piece < NPATCH) {
                const int q = piece % (CK / 8), pix = piece / (CK / 8);
                *reinterpret_cast<short8_t*>(s_x + pix * CKP + 8 * q) = rp[i];
            }
        }
#pragma unroll
        for (int i = 0; i < PW; ++i) {
            const int piece = tid + 256 * i;
            if (piece < NWT) {
                const int q = piece % (CK / 8), r = piece / (CK / 8);
                *reinterpret_cast<short8_t*>(s_w + r * CKP + 8 * q) = rw[i];
            }
        }
    };

    float4_t acc[COT / 16];
#pragma unroll
    for (int j = 0; j < COT / 16; ++j) acc[j] = {0.f, 0.f, 0.f, 0.f};
    const int m = lane & 15, kq = 8 * (lane >> 4);
    fetch(0);
    for (int kc = 0; kc < Cin; kc += CK) {
        __syncthreads();
        publish();
        __syncthreads();
        if (kc + CK < Cin) fetch(kc + CK);
#pragma unroll
        for (int tap = 0; tap < T; ++tap) {
            const int dy = KS == 3 ? tap / 3 - 1 : 0, dx = KS == 3 ? tap % 3 - 1 : 0;
            const short8_t a = *reinterpret_cast<const short8_t*>(
                s_x + ((wave + dy + h0) * PC + (m + dx + h0)) * CKP + kq);
#pragma unroll
            for (int j = 0; j < COT / 16; ++j) {
                const short8_t b = *reinterpret_cast<const short8_t*>(s_w + ((16 * j + m) * T + tap) * CKP + kq);
                acc[j] = mfma32(a, b, acc[j]);
            }
        }
    }
    // D: lane (j, i/4): column = output channel, rows = 4 consecutive pixels of this wave's row
#pragma unroll
    for (int j = 0; j < COT / 16; ++j) {
        const int co = co0 + 16 * j + m;
        if (co >= Cout) continue;
        const float bb = bias ? bias[co] : 0.0f;
        const int yy = ty0 + wave;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int xx = tx0 + 4 * (lane >> 4) + e;
            if (yy >= H || xx >= W) continue;
            const long long p = (n * H + yy) * W + xx;
            float v = acc[j][e] + bb;
            if (RELU) v = fmaxf(v, 0.0f);
            y[p * ys + yo + co] = f2bf(v);
            if (yf) yf[p * Cout + co] = v;
        }
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
// One wave per (16 output channels, 64 input channels, tap, pixel chunk).
template <int KS>
__global__ __launch_bounds__(64) void conv_wgrad_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                                        int Cout, const bf16* __restrict__ x,
                                                        int xs, int xo, int Cin, int N, int H, int W,
                                                        int chunk_pix, float* __restrict__ part,
                                                        float* __restrict__ bpart) {
    const int lane = threadIdx.x;
    const int co0 = blockIdx.x * 16, ci0 = blockIdx.y * 64;
    const int tap = blockIdx.z % (KS * KS), chunk = blockIdx.z / (KS * KS);
    const int dyy = KS == 3 ? tap / 3 - 1 : 0, dxx = KS == 3 ? tap % 3 - 1 : 0;
    const long long npix = (long long)N * H * W;
    const long long pbeg = (long long)chunk * chunk_pix;
    const long long pend = min(npix, pbeg + chunk_pix);
    float4_t acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = {0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    const int kq = 4 * (lane >> 4);
    for (long long p0 = pbeg; p0 < pend; p0 += 16) {
        short4_t a;
        short4_t b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const long long p = p0 + kq + e;
            const bool ok = p < pend;
            // A[i = co][k = pixel]
            a[e] = ok ? (short)dy[p * dys + dyo + co0 + (lane & 15)] : (short)0;
            long long src = 0;
            if (ok) {
                const int xx = (int)(p % W), yy = (int)((p / W) % H);
                const long long nn = p / ((long long)W * H);
                int sy = yy + dyy, sx = xx + dxx;
                sy = sy < 0 ? sy + H : (sy >= H ? sy - H : sy);
                sx = sx < 0 ? sx + W : (sx >= W ? sx - W : sx);
                src = ((nn * H + sy) * W + sx) * xs + xo;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ci = ci0 + 16 * j + (lane & 15);
                b[j][e] = (ok && ci < Cin) ? (short)x[src + ci] : (short)0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = mfma16(a, b[j], acc[j]);
        if (tap == 0 && blockIdx.y == 0) {
            // bias: lanes 0..15 sum dy over the 16 pixels of this step for their channel
            if (lane < 16)
                for (int k = 0; k < 16 && p0 + k < pend; ++k) bsum += bf2f(dy[(p0 + k) * dys + dyo + co0 + lane]);
        }
    }
    const int taps = KS * KS;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int ci = ci0 + 16 * j + (lane & 15);
        if (ci >= Cin) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = co0 + 4 * (lane >> 4) + e;
            part[(((long long)chunk * Cout + co) * taps + tap) * Cin + ci] = acc[j][e];
        }
    }
    if (tap == 0 && blockIdx.y == 0 && lane < 16) bpart[(long long)chunk * Cout + co0 + lane] = bsum;
}

// Deterministic sum over chunks: out[i] = sum_c part[c][i]
__global__ void sum_chunks_kernel(const float* __restrict__ part, long long n, int nchunks,
                                  float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < nchunks; ++c) s += part[(long long)c * n + i];
        out[i] = s;
    }
}

// 2x2 average pool: y[n, Y, X, c] = mean of x[n, 2Y..2Y+1, 2X..2X+1, c] (x slice xs/xo, C ch)
__global__ void avgpool_kernel(const bf16* __restrict__ x, int xs, int xo, bf16* __restrict__ y,
                               int ys, int yo, int C, int N, int H, int W) {
    const int Ho = H / 2, Wo = W / 2;
    const long long n = (long long)N * Ho * Wo * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long q = i / C;
        const int X = (int)(q % Wo), Y = (int)((q / Wo) % Ho);
        const long long nn = q / ((long long)Wo * Ho);
        const long long b = ((nn * H + 2 * Y) * W + 2 * X);
        const float s = bf2f(x[b * xs + xo + c]) + bf2f(x[(b + 1) * xs + xo + c]) +
                        bf2f(x[(b + W) * xs + xo + c]) + bf2f(x[(b + W + 1) * xs + xo + c]);
        y[q * ys + yo + c] = f2bf(0.25f * s);
    }
}

// gradient of the pool added into the input-gradient slice: dx[p] += dy[parent(p)] / 4
__global__ void avgpool_bwd_add_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                       bf16* __restrict__ dx, int dxs, int dxo, int C, int N, int H,
                                       int W) {
    const long long n = (long long)N * H * W * C;
    const int Ho = H / 2, Wo = W / 2;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long p = i / C;
        const int xx = (int)(p % W), yy = (int)((p / W) % H);
        const long long nn = p / ((long long)W * H);
        const long long q = (nn * Ho + yy / 2) * Wo + xx / 2;
        const float v = bf2f(dx[p * dxs + dxo + c]) + 0.25f * bf2f(dy[q * dys + dyo + c]);
        dx[p * dxs + dxo + c] = f2bf(v);
    }
}

// nearest 2x upsample: y[n, y, x, c] = x[n, y/2, x/2, c] (output H x W)
__global__ void upsample_kernel(const bf16* __restrict__ x, int xs, int xo, bf16* __restrict__ y,
                                int ys, int yo, int C, int N, int H, int W) {
    const long long n = (long long)N * H * W * C;
    const int Hi = H / 2, Wi = W / 2;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long p = i / C;
        const int xx = (int)(p % W), yy = (int)((p / W) % H);
        const long long nn = p / ((long long)W * H);
        y[p * ys + yo + c] = x[((nn * Hi + yy / 2) * Wi + xx / 2) * xs + xo + c];
    }
}

// gradient of the upsample: dx[q, c] = sum of dy over the 4 children of q (dx full buffer)
__global__ void upsample_bwd_kernel(const bf16* __restrict__ dy, int dys, int dyo,
                                    bf16* __restrict__ dx, int dxs, int dxo, int C, int N, int H,
                                    int W) {
    const int Ho = H / 2, Wo = W / 2;
    const long long n = (long long)N * Ho * Wo * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long q = i / C;
        const int X = (int)(q % Wo), Y = (int)((q / Wo) % Ho);
        const long long nn = q / ((long long)Wo * Ho);
        const long long b = ((nn * H + 2 * Y) * W + 2 * X);
        const float s = bf2f(dy[b * dys + dyo + c]) + bf2f(dy[(b + 1) * dys + dyo + c]) +
                        bf2f(dy[(b + W) * dys + dyo + c]) + bf2f(dy[(b + W + 1) * dys + dyo + c]);
        dx[q * dxs + dxo + c] = f2bf(s);
    }
}

// ReLU gradient in place: g *= (a > 0), a the post-activation of the same slice layout
__global__ void relu_bwd_kernel(bf16* __restrict__ g, int gs, int go, const bf16* __restrict__ a,
                                int as, int ao, int C, long long npix) {
    const long long n = npix * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long p = i / C;
        if (!(bf2f(a[p * as + ao + c]) > 0.0f)) g[p * gs + go + c] = 0;
    }
}

// pack network input: x0 (bf16, 16 channels, zero beyond cin) from FP32 NHWC [.., cin]
__global__ void pack_input_kernel(const float* __restrict__ in, int cin, bf16* __restrict__ x0,
                                  long long npix) {
    const long long n = npix * 16;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % 16);
        const long long p = i / 16;
        x0[i] = c < cin ? f2bf(in[p * cin + c]) : (bf16)0;
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

hipError_t unet_conv_fwd(int ks, bool relu, const bf16* x, int xs, int xo, int Cin, const bf16* w,
                         const float* bias, bf16* y, int ys, int yo, int Cout, float* yf, int N,
                         int H, int W, hipStream_t st) {
    // LDS-tiled MFMA kernel whenever the 16-byte pieces stay aligned, else the plain one
    const bool tiled = (Cin % 8 == 0) && (xs % 8 == 0) && (xo % 8 == 0);
    if (tiled) {
        const long long tiles = (long long)N * ((H + 3) / 4) * ((W + 15) / 16);
        const int cot = Cout <= 32 ? 32 : 64;
        dim3 grid((unsigned)tiles, (unsigned)((Cout + cot - 1) / cot));
#define LBPF_CONV(KS_, R_, C_) hipLaunchKernelGGL((conv_lds_kernel<KS_, R_, C_>), grid, dim3(256), 0, st, \
                                                  x, xs, xo, Cin, w, bias, y, ys, yo, Cout, yf, N, H, W)
        if (ks == 3) {
            if (relu) { if (cot == 32) LBPF_CONV(3, true, 32); else LBPF_CONV(3, true, 64); }
            else { if (cot == 32) LBPF_CONV(3, false, 32); else LBPF_CONV(3, false, 64); }
        } else {
            if (relu) { if (cot == 32) LBPF_CONV(1, true, 32); else LBPF_CONV(1, true, 64); }
            else { if (cot == 32) LBPF_CONV(1, false, 32); else LBPF_CONV(1, false, 64); }
        }
#undef LBPF_CONV
        return hipGetLastError();
    }
    const long long npix = (long long)N * H * W;
    dim3 grid((unsigned)((npix + 63) / 64), (unsigned)((Cout + 63) / 64));
    if (ks == 3 && relu)
        hipLaunchKernelGGL((conv_fwd_kernel<3, true>), grid, dim3(256), 0, st, x, xs, xo, Cin, w, bias, y, ys, yo, Cout, yf, N, H, W);
    else if (ks == 3)
        hipLaunchKernelGGL((conv_fwd_kernel<3, false>), grid, dim3(256), 0, st, x, xs, xo, Cin, w, bias, y, ys, yo, Cout, yf, N, H, W);
    else if (relu)
        hipLaunchKernelGGL((conv_fwd_kernel<1, true>), grid, dim3(256), 0, st, x, xs, xo, Cin, w, bias, y, ys, yo, Cout, yf, N, H, W);
    else
        hipLaunchKernelGGL((conv_fwd_kernel<1, false>), grid, dim3(256), 0, st, x, xs, xo, Cin, w, bias, y, ys, yo, Cout, yf, N, H, W);
    return hipGetLastError();
}

hipError_t unet_flip_weights(const bf16* w, bf16* wt, int Cout, int Cin, int taps, hipStream_t st) {
    hipLaunchKernelGGL(flip_weights_kernel, ew_grid((long long)Cout * Cin * taps), dim3(256), 0, st, w, wt, Cout, Cin, taps);
    return hipGetLastError();
}

hipError_t unet_conv_wgrad(int ks, const bf16* dy, int dys, int dyo, int Cout, const bf16* x, int xs,
                           int xo, int Cin, int N, int H, int W, int nchunks, float* part,
                           float* bpart, float* dw, float* db, hipStream_t st) {
    const long long npix = (long long)N * H * W;
    long long chunk = (npix + nchunks - 1) / nchunks;
    chunk = (chunk + 15) / 16 * 16;
    const int taps = ks * ks;
    dim3 grid((unsigned)(Cout / 16), (unsigned)((Cin + 63) / 64), (unsigned)(taps * nchunks));
    if (ks == 3)
        hipLaunchKernelGGL((conv_wgrad_kernel<3>), grid, dim3(64), 0, st, dy, dys, dyo, Cout, x, xs, xo, Cin, N, H, W, (int)chunk, part, bpart);
    else
        hipLaunchKernelGGL((conv_wgrad_kernel<1>), grid, dim3(64), 0, st, dy, dys, dyo, Cout, x, xs, xo, Cin, N, H, W, (int)chunk, part, bpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nw = (long long)Cout * taps * Cin;
    hipLaunchKernelGGL(sum_chunks_kernel, ew_grid(nw), dim3(256), 0, st, part, nw, nchunks, dw);
    hipLaunchKernelGGL(sum_chunks_kernel, ew_grid(Cout), dim3(256), 0, st, bpart, (long long)Cout, nchunks, db);
    return hipGetLastError();
}

hipError_t unet_avgpool(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(avgpool_kernel, ew_grid((long long)N * H * W * C / 4), dim3(256), 0, st, x, xs, xo, y, ys, yo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_avgpool_bwd_add(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(avgpool_bwd_add_kernel, ew_grid((long long)N * H * W * C), dim3(256), 0, st, dy, dys, dyo, dx, dxs, dxo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_upsample(const bf16* x, int xs, int xo, bf16* y, int ys, int yo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(upsample_kernel, ew_grid((long long)N * H * W * C), dim3(256), 0, st, x, xs, xo, y, ys, yo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_upsample_bwd(const bf16* dy, int dys, int dyo, bf16* dx, int dxs, int dxo, int C, int N, int H, int W, hipStream_t st) {
    hipLaunchKernelGGL(upsample_bwd_kernel, ew_grid((long long)N * H * W * C / 4), dim3(256), 0, st, dy, dys, dyo, dx, dxs, dxo, C, N, H, W);
    return hipGetLastError();
}
hipError_t unet_relu_bwd(bf16* g, int gs, int go, const bf16* a, int as, int ao, int C, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(relu_bwd_kernel, ew_grid(npix * C), dim3(256), 0, st, g, gs, go, a, as, ao, C, npix);
    return hipGetLastError();
}
hipError_t unet_pack_input(const float* in, int cin, bf16* x0, long long npix, hipStream_t st) {
    hipLaunchKernelGGL(pack_input_kernel, ew_grid(npix * 16), dim3(256), 0, st, in, cin, x0, npix);
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
