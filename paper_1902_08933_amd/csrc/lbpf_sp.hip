// Generalized single-phase lattice Boltzmann model with a mass source (arXiv:1902.08933,
// Sec. 2) for gfx950: kernels and the host side of the lbpf_sp_* calls of include/lbpf.h.
//
// One time step is one launch of sp_step_kernel<MODEL, FULL, BC>: every node reads its
// post-streaming populations, computes the macroscopic quantities and the force term of
// eq. (27), collides (eq. 24) and pushes the post-collision populations to x + c_i in the other
// copy (periodic wrap, or halfway bounce-back at y walls). Populations are stored in FP32 as
// deviations from a constant: g_i - w_i in the nearly incompressible model (Remark 1, whose
// equilibrium rho [w_i + s_i(u)] is w_i at rest), g_0 - rho0 in the incompressible model
// (Remark 3); every equilibrium and collision operand is then a small number and FP32 keeps
// its relative precision. The lagged quantities of the force term (div u of the previous step,
// grad p of the previous pressure) live in ping-pong planes read through the L2 cache.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbpf.h"

namespace lbpf_sp_detail {

constexpr int kQ = 9;
__device__ constexpr int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float kW0 = 4.0f / 9.0f, kWA = 1.0f / 9.0f, kWD = 1.0f / 36.0f;
__device__ __forceinline__ constexpr float wq(int q) { return q == 0 ? kW0 : (q < 5 ? kWA : kWD); }

// Workspace planes (each ny * pitch + pad floats): populations A [0, 9), B [9, 18), S, Fx, Fy,
// four history planes (nearly incompressible: u_x, u_y of the previous step, copies 0 and 1;
// incompressible with the full force term: the previous pressure, copies 0 and 1), then the
// FP64 reduction area.
constexpr int kPlaneGA = 0, kPlaneGB = 9, kPlaneS = 18, kPlaneFx = 19, kPlaneFy = 20;
constexpr int kPlaneHist = 21, kPlaneG = 25, kNumPlanes = 25, kNumPlanesR4 = 43;  // + G, 2 copies
constexpr int kRedBlocks = 1024;
constexpr long kPad = 4160;  // floats between planes, as for the two-phase solver

struct SpModel {
    int nx, ny, pitch;
    long long plane;
    int bc;
    float tau, omega, fgain;   // tau_g, 1/tau_g, 1 - 1/(2 tau_g)
    float xi_term;             // xi/(tau_g - 1/2)
    float rho0;
    int pscheme;
    float pc, ipc;             // eq. (28) with d_t p = p - p^{n-1}: c = 0.8 (tau - 1/2), 1/(1 + c)
    float drag;                // lambda: F = F_ext - lambda rho u (model 0)
    int scheme;                // model 0: 0 eq. (24), 1 Remark 4 (explicit D_i G_i)
};

__device__ __forceinline__ int wrapi(int v, int n) {
    if ((unsigned)v < (unsigned)n) return v;
    const int r = v % n;
    return r < 0 ? r + n : r;
}
template <int BC>
__device__ __forceinline__ int row_of(int y, int ny) {
    if (BC == 0) return wrapi(y, ny);
    if (y < 0) y = -1 - y;
    else if (y >= ny) y = 2 * ny - 1 - y;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// eq. (30a) of a plane at (x, y): grad z = 3 sum_{i != 0} w_i c_i z(x + c_i)
template <int BC>
__device__ __forceinline__ void grad30a(const SpModel& m, const float* __restrict__ z, int x, int y,
                                        float& gx, float& gy) {
    const int xp = wrapi(x + 1, m.nx), xm = wrapi(x - 1, m.nx);
    const long long rN = (long long)row_of<BC>(y + 1, m.ny) * m.pitch;
    const long long rC = (long long)y * m.pitch;
    const long long rS = (long long)row_of<BC>(y - 1, m.ny) * m.pitch;
    const float E = z[rC + xp], Wv = z[rC + xm], N = z[rN + x], Sv = z[rS + x];
    const float NE = z[rN + xp], NW = z[rN + xm], SE = z[rS + xp], SW = z[rS + xm];
    gx = (1.0f / 3.0f) * (E - Wv) + (1.0f / 12.0f) * ((NE - NW) + (SE - SW));
    gy = (1.0f / 3.0f) * (N - Sv) + (1.0f / 12.0f) * ((NE - SE) + (NW - SW));
}

struct Macro {
    float drho;  // rho - 1 (model 0), 0 (model 1)
    float rho, ux, uy, p;
    float axx, axy, ayy;  // bracket of eq. (27)
    float S, Fx, Fy;
};

// Macroscopic quantities and the bracket of the force term at one node (both models).
// g: deviations; hx, hy: the previous step's velocity (model 0) or hx: the previous step's
// pressure (model 1 with the full force term).
template <int MODEL, bool FULL, int BC>
__device__ __forceinline__ Macro sp_macro(const SpModel& m, const float (&g)[kQ], float S, float Fx,
                                          float Fy, const float* __restrict__ hx,
                                          const float* __restrict__ hy, int x, int y, long long c) {
    Macro r;
    r.S = S; r.Fx = Fx; r.Fy = Fy;
    const float sum = (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
    const float mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
    const float my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
    if (MODEL == 0) {
        if (m.scheme == 0) {
            // eq. (27aa) with rho~ = rho: rho = sum_i g_i + S/2 = 1 + sum_i (g_i - w_i) + S/2;
            // eq. (27a) with F = F_ext - lambda rho u, solved: rho u (1 + lambda/2) = m + F_ext/2
            r.drho = sum + 0.5f * S;
            r.rho = 1.0f + r.drho;
            const float irho = __builtin_amdgcn_rcpf(r.rho * (1.0f + 0.5f * m.drag));
            r.ux = (mx + 0.5f * Fx) * irho;
            r.uy = (my + 0.5f * Fy) * irho;
        } else {
            // Remark 4 evolves f~ itself: rho~ = sum f~, rho u = sum c f~
            r.drho = sum;
            r.rho = 1.0f + r.drho;
            const float irho = __builtin_amdgcn_rcpf(r.rho);
            r.ux = mx * irho;
            r.uy = my * irho;
        }
        Fx -= m.drag * r.rho * r.ux;
        Fy -= m.drag * r.rho * r.uy;
        r.Fx = Fx;
        r.Fy = Fy;
        r.p = r.rho * (1.0f / 3.0f);
        float dxx, dxy, dyx, dyy;
        grad30a<BC>(m, hx, x, y, dxx, dxy);
        grad30a<BC>(m, hy, x, y, dyx, dyy);
        const float divu = dxx + dyy;
        const float Q = r.rho * (1.0f / 3.0f) - m.xi_term;  // (2/d) rho c_s^2 - xi/(tau - 1/2)
        const float St = FULL ? S : 0.0f;
        r.axx = 2.0f * r.ux * Fx - r.ux * r.ux * St + Q * divu;
        r.axy = r.ux * Fy + Fx * r.uy - r.ux * r.uy * St;
        r.ayy = 2.0f * r.uy * Fy - r.uy * r.uy * St + Q * divu;
    } else {
        r.drho = 0.0f;
        r.rho = 1.0f;
        r.ux = mx + 0.5f * Fx;  // eq. (27a), rho = 1
        r.uy = my + 0.5f * Fy;
        const float Q = (1.0f / 3.0f) - m.xi_term;
        float Ftx = Fx, Fty = Fy, St = 0.0f, p1 = 0.0f;
        if (FULL) {
            float gpx, gpy;
            grad30a<BC>(m, hx, x, y, gpx, gpy);
            Ftx -= gpx;
            Fty -= gpy;
            p1 = hx[c];
            St = S;
        }
        // bracket without its d_t p I part: u F~ + F~ u - u u S + Q S I (div u = S)
        r.axx = 2.0f * r.ux * Ftx - r.ux * r.ux * St + Q * S;
        r.axy = r.ux * Fty + Ftx * r.uy - r.ux * r.uy * St;
        r.ayy = 2.0f * r.uy * Fty - r.uy * r.uy * St + Q * S;
        // eq. (28): p = 3/5 [ sum_{i!=0} g_i + S/2 + s_0(u) + (tau - 1/2) G_0 ]; s_0 = -(2/3) u^2
        const float u2 = r.ux * r.ux + r.uy * r.uy;
        float br = (sum - g[0]) + 0.5f * S - (2.0f / 3.0f) * u2;
        if (m.pscheme == 0) {
            // G_0 of eq. (27): w_0 [S - 3/2 (axx + ayy)] (c_0 = 0, (0 - I/3) : A / (2/9))
            br += (m.tau - 0.5f) * (kW0 * (S - 1.5f * (r.axx + r.ayy)));
        }
        r.p = 0.6f * br;
        if (FULL) {
            // d_t p = p - p^{n-1} enters G_0 as -3 w_0 d_t p: eq. (28) solved for p, then the
            // d_t p I part of the bracket
            r.p = (r.p + m.pc * p1) * m.ipc;
            const float dtp = r.p - p1;
            r.axx += dtp;
            r.ayy += dtp;
        }
    }
    return r;
}

template <int MODEL, bool FULL, int BC>
__global__ __launch_bounds__(256) void sp_step_kernel(SpModel m, const float* __restrict__ gin,
                                                      float* __restrict__ gout,
                                                      const float* __restrict__ Sf,
                                                      const float* __restrict__ Fxf,
                                                      const float* __restrict__ Fyf,
                                                      const float* __restrict__ hx_in,
                                                      const float* __restrict__ hy_in,
                                                      float* __restrict__ h_out0,
                                                      float* __restrict__ h_out1) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= m.nx || y >= m.ny) return;
    const long long P = m.plane, c = (long long)y * m.pitch + x;
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = gin[q * P + c];
    const Macro r = sp_macro<MODEL, FULL, BC>(m, g, Sf[c], Fxf[c], Fyf[c], hx_in, hy_in, x, y, c);
    const float ux = r.ux, uy = r.uy, u2 = ux * ux + uy * uy;
    const float omega = m.omega, fgain = m.fgain;
    const int xp = (x + 1 == m.nx) ? 0 : x + 1, xm = (x == 0) ? m.nx - 1 : x - 1;
    const int yp = (y + 1 == m.ny) ? 0 : y + 1, ym = (y == 0) ? m.ny - 1 : y - 1;
    const bool wall_top = BC == 1 && y == m.ny - 1, wall_bot = BC == 1 && y == 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const float w = wq(q);
        const int cx = kCX[q], cy = kCY[q];
        const float cu = cx * ux + cy * uy;
        const float s = w * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2);  // s_i(u) of eq. (25)
        // eq. (27): w_i [S + 3 c.F + 4.5 (c c - I/3) : A]
        const float cxx = cx * cx - (1.0f / 3.0f), cyy = cy * cy - (1.0f / 3.0f), cxy = (float)(cx * cy);
        const float G = w * (r.S + 3.0f * (cx * r.Fx + cy * r.Fy) +
                             4.5f * (cxx * r.axx + 2.0f * cxy * r.axy + cyy * r.ayy));
        // equilibrium deviations: model 0, rho (w_i + s_i) - w_i = (rho - 1) w_i + rho s_i;
        // model 1, eq. (25) minus rho0 at i = 0: 3 p (w_i - [i = 0]) + s_i
        float geq;
        if (MODEL == 0) geq = r.drho * w + r.rho * s;
        else geq = 3.0f * r.p * (q == 0 ? (w - 1.0f) : w) + s;
        // eq. (24), in deviations (the constant offset cancels)
        const float gst = g[q] - (g[q] - geq) * omega + fgain * G;
        int dx = cx > 0 ? xp : (cx < 0 ? xm : x);
        int dy = cy > 0 ? yp : (cy < 0 ? ym : y);
        int dq = q;
        if ((cy > 0 && wall_top) || (cy < 0 && wall_bot)) {
            dx = x;
            dy = y;
            dq = kOpp[q];
        }
        gout[dq * P + (long long)dy * m.pitch + dx] = gst;
    }
    if (MODEL == 0) {
        h_out0[c] = ux;
        h_out1[c] = uy;
    } else if (FULL) {
        h_out0[c] = r.p;  // only the full force term reads the pressure history
    }
}

// Remark 4 (nearly incompressible model): first pass, the force distribution G_i(x, t) of every
// node (eq. 27, with the macroscopics of f~) into the G planes, and the velocity into the
// history for the next step's div u.
template <bool FULL, int BC>
__global__ __launch_bounds__(256) void sp_r4_force_kernel(SpModel m, const float* __restrict__ gin,
                                                          const float* __restrict__ Sf,
                                                          const float* __restrict__ Fxf,
                                                          const float* __restrict__ Fyf,
                                                          const float* __restrict__ hx_in,
                                                          const float* __restrict__ hy_in,
                                                          float* __restrict__ h_out0,
                                                          float* __restrict__ h_out1,
                                                          float* __restrict__ Gout) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= m.nx || y >= m.ny) return;
    const long long P = m.plane, c = (long long)y * m.pitch + x;
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = gin[q * P + c];
    const Macro r = sp_macro<0, FULL, BC>(m, g, Sf[c], Fxf[c], Fyf[c], hx_in, hy_in, x, y, c);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int cx = kCX[q], cy = kCY[q];
        const float cxx = cx * cx - (1.0f / 3.0f), cyy = cy * cy - (1.0f / 3.0f), cxy = (float)(cx * cy);
        Gout[q * P + c] = wq(q) * (r.S + 3.0f * (cx * r.Fx + cy * r.Fy) +
                                   4.5f * (cxx * r.axx + 2.0f * cxy * r.axy + cyy * r.ayy));
    }
    h_out0[c] = r.ux;
    h_out1[c] = r.uy;
}

// Remark 4, second pass: f~* = f~ - (f~ - f^eq)/tau + G_i(x, t) + [G_i(x + c_i, t) - G_i(x, t-1)]/2
// and push to x + c_i. G_i(x + c_i) across a wall link is G_i(x); before the first step
// G(t-1) = G(t) (Gprev == Gcur).
template <int BC>
__global__ __launch_bounds__(256) void sp_r4_collide_kernel(SpModel m, const float* __restrict__ gin,
                                                            float* __restrict__ gout,
                                                            const float* __restrict__ Gcur,
                                                            const float* __restrict__ Gprev) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= m.nx || y >= m.ny) return;
    const long long P = m.plane, c = (long long)y * m.pitch + x;
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = gin[q * P + c];
    const float sum = (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
    const float mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
    const float my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
    const float drho = sum, rho = 1.0f + drho, irho = __builtin_amdgcn_rcpf(rho);
    const float ux = mx * irho, uy = my * irho, u2 = ux * ux + uy * uy;
    const int xp = (x + 1 == m.nx) ? 0 : x + 1, xm = (x == 0) ? m.nx - 1 : x - 1;
    const int yp = (y + 1 == m.ny) ? 0 : y + 1, ym = (y == 0) ? m.ny - 1 : y - 1;
    const bool wall_top = BC == 1 && y == m.ny - 1, wall_bot = BC == 1 && y == 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const float w = wq(q);
        const int cx = kCX[q], cy = kCY[q];
        const float cu = cx * ux + cy * uy;
        const float geq = drho * w + rho * w * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2);
        int dx = cx > 0 ? xp : (cx < 0 ? xm : x);
        int dy = cy > 0 ? yp : (cy < 0 ? ym : y);
        const bool wall = (cy > 0 && wall_top) || (cy < 0 && wall_bot);
        const long long cn = wall ? c : (long long)dy * m.pitch + dx;
        const float Gc = Gcur[q * P + c], Gn = Gcur[q * P + cn], Gp = Gprev[q * P + c];
        const float gst = g[q] - (g[q] - geq) * m.omega + Gc + 0.5f * (Gn - Gp);
        int dq = q;
        if (wall) {
            dx = x;
            dy = y;
            dq = kOpp[q];
        }
        gout[dq * P + (long long)dy * m.pitch + dx] = gst;
    }
}

// Macroscopic field of the current state (no collision): 0 rho, 1 ux, 2 uy, 3 p
template <int MODEL, bool FULL, int BC>
__global__ __launch_bounds__(256) void sp_field_kernel(SpModel m, const float* __restrict__ gin,
                                                       const float* __restrict__ Sf,
                                                       const float* __restrict__ Fxf,
                                                       const float* __restrict__ Fyf,
                                                       const float* __restrict__ hx_in,
                                                       const float* __restrict__ hy_in, int field,
                                                       float* __restrict__ dst) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= m.nx || y >= m.ny) return;
    const long long P = m.plane, c = (long long)y * m.pitch + x;
    float g[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = gin[q * P + c];
    const Macro r = sp_macro<MODEL, FULL, BC>(m, g, Sf[c], Fxf[c], Fyf[c], hx_in, hy_in, x, y, c);
    const float v = field == 0 ? r.rho : (field == 1 ? r.ux : (field == 2 ? r.uy : r.p));
    dst[(long long)y * m.nx + x] = v;
}

// Equilibrium initial state and histories from the initial fields
__global__ __launch_bounds__(256) void sp_init_kernel(SpModel m, int model, const float* a0,
                                                      const float* ux0, const float* uy0,
                                                      const float* S, const float* Fx,
                                                      const float* Fy, float* __restrict__ g,
                                                      float* __restrict__ Sf, float* __restrict__ Fxf,
                                                      float* __restrict__ Fyf,
                                                      float* __restrict__ hist) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= m.nx || y >= m.ny) return;
    const long long P = m.plane, c = (long long)y * m.pitch + x, i = (long long)y * m.nx + x;
    const float a = a0 ? a0[i] : (model == 0 ? 1.0f : 0.0f);
    const float ux = ux0 ? ux0[i] : 0.0f, uy = uy0 ? uy0[i] : 0.0f, u2 = ux * ux + uy * uy;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const float w = wq(q);
        const float cu = kCX[q] * ux + kCY[q] * uy;
        const float s = w * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2);
        // model 0: rho (w + s) - w; model 1: eq. (25) minus rho0 at i = 0
        g[q * P + c] = model == 0 ? (a - 1.0f) * w + a * s : 3.0f * a * (q == 0 ? (w - 1.0f) : w) + s;
    }
    Sf[c] = S ? S[i] : 0.0f;
    Fxf[c] = Fx ? Fx[i] : 0.0f;
    Fyf[c] = Fy ? Fy[i] : 0.0f;
    if (model == 0) {
        hist[c] = ux;          // u_x, copy 0
        hist[2 * P + c] = uy;  // u_y, copy 0
    } else {
        hist[c] = a;  // pressure, copy 0
    }
}

// FP64 partial sums per block: rho~ = sum_i g_i + S/2 (plus 1 per node in model 0, whose
// populations are stored as g_i - w_i), rho u_x, rho u_y; then one fixed-order final pass.
template <int MODEL>
__global__ __launch_bounds__(256) void sp_sum_partial_kernel(SpModel m, const float* __restrict__ g,
                                                             const float* __restrict__ Sf,
                                                             const float* __restrict__ Fxf,
                                                             const float* __restrict__ Fyf,
                                                             double* __restrict__ part) {
    __shared__ double sh[3][4];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const long long n = (long long)m.nx * m.ny, P = m.plane;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % m.nx), y = (int)(k / m.nx);
        const long long c = (long long)y * m.pitch + x;
        double s = 0.0, mx = 0.0, my = 0.0;
        for (int q = 0; q < kQ; ++q) {
            const double v = (double)g[q * P + c];
            s += v;
            mx += kCX[q] * v;
            my += kCY[q] * v;
        }
        const double S = Sf[c];
        if (MODEL == 0 && m.scheme == 1) {
            // Remark 4: rho~ = sum f~, rho u = sum c f~
            a0 += 1.0 + s;
            a1 += mx;
            a2 += my;
        } else {
            a0 += (MODEL == 0 ? 1.0 : (double)m.rho0) + s + 0.5 * S;
            // rho u = (sum_i c_i g_i + F_ext/2) / (1 + lambda/2) (eq. 27a; rho = 1 in model 1)
            const double d = 1.0 + 0.5 * (double)m.drag;
            a1 += (mx + 0.5 * (double)Fxf[c]) / d;
            a2 += (my + 0.5 * (double)Fyf[c]) / d;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o);
        a1 += __shfl_xor(a1, o);
        a2 += __shfl_xor(a2, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { sh[0][wv] = a0; sh[1][wv] = a1; sh[2][wv] = a2; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        part[k * kRedBlocks + blockIdx.x] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
    }
}

__global__ void sp_sum_final_kernel(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[threadIdx.x * kRedBlocks + b];
        out[threadIdx.x] = s;
    }
}

}  // namespace lbpf_sp_detail

using namespace lbpf_sp_detail;

struct lbpf_sp {
    lbpf_sp_params params;
    SpModel m;
    char* ws;
    size_t ws_bytes;
    hipStream_t stream;
    int cur;        // population copy holding the current state
    int64_t step;
    bool initialized;
    std::string err;
};

static thread_local std::string g_sp_create_err;

static lbpf_status spfail(lbpf_sp* s, lbpf_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_sp_create_err = buf;
    return st;
}

static const char* sp_validate(const lbpf_sp_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
    if (p->nx >= (1 << 24) || p->ny >= (1 << 24)) return "nx and ny must be below 2^24";
    if (p->model != LBPF_SP_NEARLY_INCOMPRESSIBLE && p->model != LBPF_SP_INCOMPRESSIBLE) return "unknown model";
    if (p->pscheme != 0 && p->pscheme != 1) return "pscheme must be 0 (eq. 28) or 1 (eq. 29)";
    if (p->bc != LBPF_BC_PERIODIC && p->bc != LBPF_BC_WALLS_Y) return "unknown bc";
    if (!(p->nu > 0.0) || !std::isfinite(p->nu)) return "nu must be > 0";
    if (!std::isfinite(p->xi) || p->xi < 0.0) return "xi must be finite and >= 0";
    if (!std::isfinite(p->rho0)) return "rho0 must be finite";
    if (!std::isfinite(p->drag) || p->drag < 0.0) return "drag must be finite and >= 0";
    if (p->drag != 0.0 && p->model != LBPF_SP_NEARLY_INCOMPRESSIBLE) return "drag is defined for the nearly incompressible model";
    if (p->scheme != 0 && p->scheme != 1) return "scheme must be 0 (eq. 24) or 1 (Remark 4)";
    if (p->scheme == 1 && p->model != LBPF_SP_NEARLY_INCOMPRESSIBLE) return "Remark 4's scheme is defined for the nearly incompressible model";
    const long long pitch = (p->nx + 63) / 64 * 64;
    if ((long long)p->ny * pitch + kPad >= (1LL << 30)) return "grid too large (a plane must hold fewer than 2^30 floats)";
    return nullptr;
}

static long long sp_plane(const lbpf_sp_params* p) { return (long long)p->ny * ((p->nx + 63) / 64 * 64) + kPad; }

static int sp_num_planes(const lbpf_sp_params* p) { return p->scheme == 1 ? kNumPlanesR4 : kNumPlanes; }

static size_t sp_ws_bytes(const lbpf_sp_params* p) {
    return (size_t)sp_plane(p) * sp_num_planes(p) * sizeof(float) + (size_t)(3 * kRedBlocks + 8) * sizeof(double);
}

static float* sp_plane_ptr(lbpf_sp* s, int k) { return reinterpret_cast<float*>(s->ws) + (size_t)k * s->m.plane; }
static double* sp_red(lbpf_sp* s) {
    return reinterpret_cast<double*>(s->ws + (size_t)s->m.plane * sp_num_planes(&s->params) * sizeof(float));
}

// History planes at step n: the previous step's velocity (nearly incompressible) or pressure
// (incompressible, full force term) is copy (n & 1), the new one goes into the other copy;
// lbpf_sp_init fills copy 0 with the initial fields.
struct SpHist {
    const float *hx, *hy;
    float *o0, *o1;
};
static SpHist sp_hist(lbpf_sp* s) {
    SpHist h{};
    float* H = sp_plane_ptr(s, kPlaneHist);
    const long long P = s->m.plane;
    if (s->params.model == LBPF_SP_NEARLY_INCOMPRESSIBLE) {
        // copy k of the velocity: u_x in history plane k, u_y in plane 2 + k
        const int a = (int)(s->step & 1), b = 1 - a;
        h.hx = H + (size_t)a * P;
        h.hy = H + (size_t)(2 + a) * P;
        h.o0 = H + (size_t)b * P;
        h.o1 = H + (size_t)(2 + b) * P;
    } else {
        const int a = (int)(s->step & 1), b = 1 - a;
        h.hx = H + (size_t)a * P;  // p^{n-1}
        h.hy = h.hx;
        h.o0 = H + (size_t)b * P;  // p^n
        h.o1 = nullptr;
    }
    return h;
}

template <int MODEL, bool FULL, int BC>
static void sp_launch_step(lbpf_sp* s, const SpHist& h, dim3 grid) {
    const int a = s->cur, b = 1 - a;
    hipLaunchKernelGGL((sp_step_kernel<MODEL, FULL, BC>), grid, dim3(256), 0, s->stream, s->m,
                       sp_plane_ptr(s, a ? kPlaneGB : kPlaneGA), sp_plane_ptr(s, b ? kPlaneGB : kPlaneGA),
                       sp_plane_ptr(s, kPlaneS), sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy),
                       h.hx, h.hy, h.o0, h.o1);
}
// Remark 4: G of this step into G copy (n & 1), then the collision reading it and the other copy
template <bool FULL, int BC>
static void sp_launch_r4(lbpf_sp* s, const SpHist& h, dim3 grid) {
    const int a = s->cur, b = 1 - a;
    const int gc = (int)(s->step & 1);
    float* Gc = sp_plane_ptr(s, kPlaneG + 9 * gc);
    const float* Gp = s->step == 0 ? Gc : sp_plane_ptr(s, kPlaneG + 9 * (1 - gc));
    const float* gin = sp_plane_ptr(s, a ? kPlaneGB : kPlaneGA);
    hipLaunchKernelGGL((sp_r4_force_kernel<FULL, BC>), grid, dim3(256), 0, s->stream, s->m, gin,
                       sp_plane_ptr(s, kPlaneS), sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy),
                       h.hx, h.hy, h.o0, h.o1, Gc);
    hipLaunchKernelGGL((sp_r4_collide_kernel<BC>), grid, dim3(256), 0, s->stream, s->m, gin,
                       sp_plane_ptr(s, b ? kPlaneGB : kPlaneGA), (const float*)Gc, Gp);
}

template <int MODEL, bool FULL, int BC>
static void sp_launch_field(lbpf_sp* s, const SpHist& h, dim3 grid, int field, float* dst) {
    hipLaunchKernelGGL((sp_field_kernel<MODEL, FULL, BC>), grid, dim3(256), 0, s->stream, s->m,
                       sp_plane_ptr(s, s->cur ? kPlaneGB : kPlaneGA), sp_plane_ptr(s, kPlaneS),
                       sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy), h.hx, h.hy, field, dst);
}

// dispatch over the compile-time switches
#define LBPF_SP_DISPATCH(FN, ...)                                                              \
    do {                                                                                        \
        const bool full_ = s->params.full != 0;                                                 \
        const int bc_ = s->params.bc;                                                           \
        if (s->params.model == 0) {                                                             \
            if (full_) { if (bc_) FN<0, true, 1>(__VA_ARGS__); else FN<0, true, 0>(__VA_ARGS__); }   \
            else { if (bc_) FN<0, false, 1>(__VA_ARGS__); else FN<0, false, 0>(__VA_ARGS__); }       \
        } else {                                                                                \
            if (full_) { if (bc_) FN<1, true, 1>(__VA_ARGS__); else FN<1, true, 0>(__VA_ARGS__); }   \
            else { if (bc_) FN<1, false, 1>(__VA_ARGS__); else FN<1, false, 0>(__VA_ARGS__); }       \
        }                                                                                       \
    } while (0)

static dim3 sp_grid(const lbpf_sp* s) { return dim3((s->m.nx + 63) / 64, (s->m.ny + 3) / 4); }

extern "C" {

lbpf_status lbpf_sp_workspace_size(const lbpf_sp_params* params, size_t* bytes) {
    if (const char* why = sp_validate(params)) return spfail(nullptr, LBPF_E_INVALID, "%s", why);
    if (!bytes) return spfail(nullptr, LBPF_E_INVALID, "bytes is NULL");
    *bytes = sp_ws_bytes(params);
    return LBPF_OK;
}

lbpf_status lbpf_sp_create(const lbpf_sp_params* params, void* workspace, size_t workspace_bytes,
                           void* hip_stream, lbpf_sp** out) {
    if (!out) return spfail(nullptr, LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (const char* why = sp_validate(params)) return spfail(nullptr, LBPF_E_INVALID, "%s", why);
    if (!workspace) return spfail(nullptr, LBPF_E_INVALID, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return spfail(nullptr, LBPF_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < sp_ws_bytes(params))
        return spfail(nullptr, LBPF_E_NOMEM, "workspace of %zu bytes, %zu needed", workspace_bytes, sp_ws_bytes(params));
    lbpf_sp* s = new (std::nothrow) lbpf_sp();
    if (!s) return spfail(nullptr, LBPF_E_NOMEM, "host allocation failed");
    s->params = *params;
    SpModel& m = s->m;
    m.nx = params->nx;
    m.ny = params->ny;
    m.pitch = (params->nx + 63) / 64 * 64;
    m.plane = sp_plane(params);
    m.bc = params->bc;
    const double tau = params->nu * 3.0 + 0.5;
    m.tau = (float)tau;
    m.omega = (float)(1.0 / tau);
    m.fgain = (float)(1.0 - 0.5 / tau);
    m.xi_term = (float)(params->xi / (tau - 0.5));
    m.rho0 = (float)params->rho0;
    m.pscheme = params->pscheme;
    const double pc = params->pscheme == 0 ? 0.8 * (tau - 0.5) : 0.0;  // (3/5)(tau - 1/2)(4/9) 3
    m.pc = (float)pc;
    m.ipc = (float)(1.0 / (1.0 + pc));
    m.drag = (float)params->drag;
    m.scheme = params->scheme;
    s->ws = static_cast<char*>(workspace);
    s->ws_bytes = workspace_bytes;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->cur = 0;
    s->step = 0;
    s->initialized = false;
    *out = s;
    return LBPF_OK;
}

lbpf_status lbpf_sp_init(lbpf_sp* s, const float* a0, const float* ux0, const float* uy0,
                         const float* S, const float* Fx, const float* Fy) {
    if (!s) return LBPF_E_INVALID;
    s->err.clear();
    s->cur = 0;
    s->step = 0;
    hipLaunchKernelGGL(sp_init_kernel, sp_grid(s), dim3(256), 0, s->stream, s->m, s->params.model, a0,
                       ux0, uy0, S, Fx, Fy, sp_plane_ptr(s, kPlaneGA), sp_plane_ptr(s, kPlaneS),
                       sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy), sp_plane_ptr(s, kPlaneHist));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spfail(s, LBPF_E_HIP, "init kernel: %s", hipGetErrorString(e));
    s->initialized = true;
    return LBPF_OK;
}

lbpf_status lbpf_sp_step(lbpf_sp* s, int64_t nsteps) {
    if (!s) return LBPF_E_INVALID;
    s->err.clear();
    if (!s->initialized) return spfail(s, LBPF_E_STATE, "lbpf_sp_init has not been called");
    if (nsteps < 0) return spfail(s, LBPF_E_INVALID, "nsteps must be >= 0");
    const dim3 grid = sp_grid(s);
    for (int64_t t = 0; t < nsteps; ++t) {
        const SpHist h = sp_hist(s);
        if (s->params.scheme == 1) {
            if (s->params.full) {
                if (s->params.bc) sp_launch_r4<true, 1>(s, h, grid); else sp_launch_r4<true, 0>(s, h, grid);
            } else {
                if (s->params.bc) sp_launch_r4<false, 1>(s, h, grid); else sp_launch_r4<false, 0>(s, h, grid);
            }
        } else {
            LBPF_SP_DISPATCH(sp_launch_step, s, h, grid);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return spfail(s, LBPF_E_HIP, "step kernel: %s", hipGetErrorString(e));
        s->cur = 1 - s->cur;
        s->step += 1;
    }
    return LBPF_OK;
}

lbpf_status lbpf_sp_read(lbpf_sp* s, int32_t field, float* dst) {
    if (!s) return LBPF_E_INVALID;
    s->err.clear();
    if (!s->initialized) return spfail(s, LBPF_E_STATE, "lbpf_sp_init has not been called");
    if (field < 0 || field > 3 || !dst) return spfail(s, LBPF_E_INVALID, "field must be 0..3 and dst non-NULL");
    const SpHist h = sp_hist(s);
    LBPF_SP_DISPATCH(sp_launch_field, s, h, sp_grid(s), field, dst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spfail(s, LBPF_E_HIP, "field kernel: %s", hipGetErrorString(e));
    return LBPF_OK;
}

lbpf_status lbpf_sp_sums(lbpf_sp* s, double* out3) {
    if (!s) return LBPF_E_INVALID;
    s->err.clear();
    if (!s->initialized) return spfail(s, LBPF_E_STATE, "lbpf_sp_init has not been called");
    if (!out3) return spfail(s, LBPF_E_INVALID, "out3 is NULL");
    const long long n = (long long)s->m.nx * s->m.ny;
    int nb = (int)((n + 1023) / 1024);
    if (nb > kRedBlocks) nb = kRedBlocks;
    double* red = sp_red(s);
    const float* g = sp_plane_ptr(s, s->cur ? kPlaneGB : kPlaneGA);
    if (s->params.model == 0)
        hipLaunchKernelGGL(sp_sum_partial_kernel<0>, dim3(nb), dim3(256), 0, s->stream, s->m, g,
                           sp_plane_ptr(s, kPlaneS), sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy), red);
    else
        hipLaunchKernelGGL(sp_sum_partial_kernel<1>, dim3(nb), dim3(256), 0, s->stream, s->m, g,
                           sp_plane_ptr(s, kPlaneS), sp_plane_ptr(s, kPlaneFx), sp_plane_ptr(s, kPlaneFy), red);
    hipLaunchKernelGGL(sp_sum_final_kernel, dim3(1), dim3(64), 0, s->stream, red, nb, red + 3 * kRedBlocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out3, red + 3 * kRedBlocks, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return spfail(s, LBPF_E_HIP, "sums: %s", hipGetErrorString(e));
    return LBPF_OK;
}

int64_t lbpf_sp_step_count(const lbpf_sp* s) { return s ? s->step : -1; }

lbpf_status lbpf_sp_destroy(lbpf_sp* s) {
    delete s;
    return LBPF_OK;
}

const char* lbpf_sp_last_error(const lbpf_sp* s) { return s ? s->err.c_str() : g_sp_create_err.c_str(); }

}  // extern "C"
