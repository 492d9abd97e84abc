// Per-node arithmetic of one time step of the phase-field LB model (arXiv:1902.08933, Sec. 3),
// in FP32, shared by every kernel that steps the solver. The caller gathers the populations of
// the node and the stencil values around it; cell_update computes the macroscopic quantities
// and, when colliding, the post-collision populations and their streaming destinations.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbpf_model.hpp"

namespace lbpf {

// D2Q9 (Sec. 2.2, listed after eq. 25)
__device__ constexpr int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float kW0 = 4.0f / 9.0f, kWA = 1.0f / 9.0f, kWD = 1.0f / 36.0f;
// 3 w_i in the parts of the collision odd in c_i, which carry the momentum: FP32 values whose
// lattice sum 2 (3 w_A) + 4 (3 w_D) is exactly 1. The nearest FP32 values of 1/3 and 1/12 sum to
// 1 + 3e-8, which multiplies the momentum by 1 + 3e-8 omega every step; near tau = 1/2 that
// compounds into a steady-state velocity ~0.3 % above the FP64 one.
constexpr float k3WA = 0x1.555556p-2f, k3WD = 0x1.555554p-4f;
static_assert(2.0 * (double)k3WA + 4.0 * (double)k3WD == 1.0, "odd-part weights must sum to 1");
__device__ __forceinline__ constexpr float wgt(int q) { return q == 0 ? kW0 : (q < 5 ? kWA : kWD); }

// Error-free transformation of a sum (Knuth): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Element `off` of plane `q` of a plane array. The plane base is the same for every lane
// (scalar registers) and the per-lane part is a 32-bit byte offset (a plane holds fewer than
// 2^30 floats), so loads and stores use the scalar-base addressing form with no 64-bit
// address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T* pl(T* base, long long plane, int q, unsigned off) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(base + q * plane) + (off << 2));
}

// 1/x with the hardware reciprocal (relative error within 1 ulp)
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int wrap(int v, int n) {
    if ((unsigned)v < (unsigned)n) return v;
    if (v < 0 && v >= -n) return v + n;
    if (v >= n && v < 2 * n) return v - n;
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Offset of node (x, y) in a plane, y * pitch + x, with the full-rate 24-bit multiply (grid
// sides are below 2^24 and a plane holds fewer than 2^30 nodes).
__device__ __forceinline__ unsigned node_off(int y, int pitch, int x) {
    return (unsigned)__umul24(y, pitch) + (unsigned)x;
}

// Row read for a stencil ghost: periodic wrap, or the mirror image about a wall half a cell
// outside the first/last fluid row (clamped for rows that no active node reads).
// BC: 0 periodic in y, 1 walls at y = -1/2 and y = ny - 1/2.
template <int BC>
__device__ __forceinline__ int src_row(int y, int ny) {
    if (BC == 0) return wrap(y, ny);
    if (y < 0) y = -1 - y;
    else if (y >= ny) y = 2 * ny - 1 - y;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// phi = sum_i h_i (eq. 18) as an unevaluated FP32 pair, from the ten stored h planes
// (h_0 hi, h_1..h_8, h_0 lo)
__device__ __forceinline__ void phi_pair(const float (&h)[kHPlanes], float& hi, float& lo) {
    float s = 0.0f;
#pragma unroll
    for (int q = 1; q <= 8; ++q) s += h[q];
    float e;
    two_sum(h[0], s, hi, e);
    lo = h[kH0Lo] + e;
}

// mu of eq. (8) at a node from the phi pairs of the node (c) and its neighbours, with the
// Laplacian of eq. (30b) taken on differences of pairs so that phi keeps its full precision.
// Rows S, C, N are offsets of the rows below, at and above the node; px is the column.
__device__ __forceinline__ float mu_at(const Model& m, const float* phh, const float* phl, int rS,
                                       int rC, int rN, int px) {
    const int c = rC + px;
    const float ch = phh[c], cl = phl[c];
    auto d = [&](int i) { return (phh[i] - ch) + (phl[i] - cl); };
    const float axes = (d(c + 1) + d(c - 1)) + (d(rN + px) + d(rS + px));
    const float diag = (d(rN + px + 1) + d(rN + px - 1)) + (d(rS + px + 1) + d(rS + px - 1));
    const float lap = (2.0f / 3.0f) * axes + (1.0f / 6.0f) * diag;
    const float a = ch + cl, b = (ch - 1.0f) + cl, cc = (ch - 0.5f) + cl;
    return m.beta4 * a * b * cc - m.kappa * lap;
}

struct Stencil {
    float phh, phl;        // phi pair at the node
    float gphix, gphiy;    // grad phi, eq. (30a)
    float mu, gmux, gmuy;  // mu and grad mu
    float lapmu;           // lap mu, eq. (30b)
    float gpx, gpy;        // grad of the previous step's pressure
};

// Stencil values at a node from LDS rows: phi pairs (rows pS, pC, pN, column px), mu and the
// previous pressure (rows mS, mC, mN, column mx). eq. (30a):
// grad z = (z_E - z_W)/3 + (z_NE - z_NW + z_SE - z_SW)/12 and likewise in y.
__device__ __forceinline__ Stencil gather(const float* phh, const float* phl, int pS, int pC,
                                          int pN, int px, const float* smu, const float* sp,
                                          int mS, int mC, int mN, int mx) {
    Stencil s;
    s.phh = phh[pC + px];
    s.phl = phl[pC + px];
    auto dp = [&](int a, int b) { return (phh[a] - phh[b]) + (phl[a] - phl[b]); };
    s.gphix = (1.0f / 3.0f) * dp(pC + px + 1, pC + px - 1)
            + (1.0f / 12.0f) * (dp(pN + px + 1, pN + px - 1) + dp(pS + px + 1, pS + px - 1));
    s.gphiy = (1.0f / 3.0f) * dp(pN + px, pS + px)
            + (1.0f / 12.0f) * (dp(pN + px + 1, pS + px + 1) + dp(pN + px - 1, pS + px - 1));
    auto grad = [&](const float* z, float& gx, float& gy) {
        gx = (1.0f / 3.0f) * (z[mC + mx + 1] - z[mC + mx - 1])
           + (1.0f / 12.0f) * ((z[mN + mx + 1] - z[mN + mx - 1]) + (z[mS + mx + 1] - z[mS + mx - 1]));
        gy = (1.0f / 3.0f) * (z[mN + mx] - z[mS + mx])
           + (1.0f / 12.0f) * ((z[mN + mx + 1] - z[mS + mx + 1]) + (z[mN + mx - 1] - z[mS + mx - 1]));
    };
    grad(smu, s.gmux, s.gmuy);
    grad(sp, s.gpx, s.gpy);
    const float mu = smu[mC + mx];
    s.mu = mu;
    s.lapmu = (2.0f / 3.0f) * (((smu[mC + mx + 1] - mu) + (smu[mC + mx - 1] - mu))
                             + ((smu[mN + mx] - mu) + (smu[mS + mx] - mu)))
            + (1.0f / 6.0f) * (((smu[mN + mx + 1] - mu) + (smu[mN + mx - 1] - mu))
                             + ((smu[mS + mx + 1] - mu) + (smu[mS + mx - 1] - mu)));
    return s;
}

// One node: closure, force, velocity (eq. 27a), mass source, F~, eq. (28) pressure, then either
// the macroscopic fields (COLLIDE = false: phi, rho, ux, uy, p, mu written to `fields` planes)
// or both BGK collisions (eq. 24, eq. 10 with eqs. 33, 34, 11, 14) with push-streaming into
// fout / hout, the new pressure into pout and (phi u) into phiu. f holds f_1..f_8, h the ten h
// planes, pu the previous (phi u). `cell` is the node's offset in a plane.
template <bool COLLIDE, int BC>
__device__ __forceinline__ void cell_update(const Model& m, int x, int y, unsigned cell,
                                            const float (&f8)[kFPlanes], const float (&h10)[kHPlanes],
                                            const float (&pu)[2], const Stencil& st,
                                            float* __restrict__ fout, float* __restrict__ hout,
                                            float* __restrict__ pout, float* __restrict__ phiu,
                                            float* __restrict__ fields) {
    const long long P = m.plane;
    float f[9], h[9];
#pragma unroll
    for (int q = 1; q <= 8; ++q) f[q] = f8[q - 1];
    float hs = 0.0f;
#pragma unroll
    for (int q = 1; q <= 8; ++q) {
        h[q] = h10[q];
        hs += h[q];
    }
    const float mu = st.mu, gphix = st.gphix, gphiy = st.gphiy;

    // closure: eq. (3aa), forces
    const float phi = st.phh + st.phl;
    const float phic = m.clamp ? fminf(fmaxf(phi, 0.0f), 1.0f) : phi;
    const float rho = m.rhoB + m.drho * phic;
    float Fx, Fy;
    if (m.fsurf == 0) { Fx = mu * gphix; Fy = mu * gphiy; }
    else { Fx = -phi * st.gmux; Fy = -phi * st.gmuy; }
    Fx += m.fx;
    Fy += m.fy - (rho - m.rhoA) * m.grav;
    // eq. (27a): u = (sum_i c_i g_i + F/2) / rho
    const float mx = ((f[1] - f[3]) + (f[5] - f[7])) + (f[8] - f[6]);
    const float my = ((f[2] - f[4]) + (f[5] - f[7])) + (f[6] - f[8]);
    const float irho = rcp(rho);
    const float ux = (mx + 0.5f * Fx) * irho, uy = (my + 0.5f * Fy) * irho;
    // mass source: S1 = -gamma M lap(mu) (quasi-incompressible) or 0; S = u.grad(rho) + rho S1
    const float S1 = (m.variant == 0) ? -m.gammaM * st.lapmu : 0.0f;
    const float grx = m.drho * gphix, gry = m.drho * gphiy;
    const float rS1 = rho * S1;
    const float S = (ux * grx + uy * gry) + rS1;
    // F~ = F - grad(p - rho c_s^2) with the previous step's pressure
    const float Ftx = Fx - st.gpx + (1.0f / 3.0f) * grx, Fty = Fy - st.gpy + (1.0f / 3.0f) * gry;
    const float uFt = ux * Ftx + uy * Fty;
    // tau_g from nu(phi): nu = c_s^2 (tau_g - 1/2)
    float nu;
    if (m.visc == 0) nu = rcp(phic * (m.inv_nuA - m.inv_nuB) + m.inv_nuB);
    else nu = ((phi >= 0.5f) ? m.muA : m.muB) * irho;
    const float tau_g = 3.0f * nu + 0.5f;
    // eq. (28): p = 3/5 [ sum_{i!=0} g_i + S/2 + rho s_0(u) + (tau_g - 1/2) G_0 ]
    const float u2 = ux * ux + uy * uy;
    const float sumf = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
    float bracket = sumf + 0.5f * S - (2.0f / 3.0f) * rho * u2;
    if (m.pscheme == 0) {
        // eq. (34) at i = 0: G_0 = w_0 (S - u.F~/c_s^2 - rho S1)
        bracket += (tau_g - 0.5f) * (kW0 * (S - 3.0f * uFt - rS1));
    } else if (m.pscheme == 1) {
        const float uFp = ux * (Fx - st.gpx) + uy * (Fy - st.gpy);
        bracket += (tau_g - 0.5f) * (kW0 * (0.5f * rS1 - 3.0f * uFp));
    }
    const float p = 0.6f * bracket;
    const float phiux = phi * ux, phiuy = phi * uy;

    if constexpr (!COLLIDE) {
        *pl(fields, P, 0, cell) = phi;
        *pl(fields, P, 1, cell) = rho;
        *pl(fields, P, 2, cell) = ux;
        *pl(fields, P, 3, cell) = uy;
        *pl(fields, P, 4, cell) = p;
        *pl(fields, P, 5, cell) = mu;
    } else {
        const int nx = m.nx, ny = m.ny, pitch = m.pitch;
        const float omega = rcp(tau_g), om1 = 1.0f - omega;
        const float fgain = 1.0f - 0.5f * omega;
        const float emu = m.eta * mu;
        const float dpx = phiux - pu[0], dpy = phiuy - pu[1];
        const float rcoef = 3.0f * m.src_coef;
        const float ith = m.inv_tau_h, ith1 = 1.0f - ith;
        // Both collisions, eq. (24) and eq. (10), written as g* = (1 - omega) g + omega g^eq
        // + (1 - omega/2) G and h* = (1 - 1/tau_h) h + h^eq/tau_h + R, and taken by pairs of
        // opposite directions (c_j = -c_i): the parts of G_i (eq. 34 expanded for d = 2),
        // g_i^eq (eq. 33, i != 0) and h_i^eq (eq. 11, i != 0) that are even in c_i are shared by
        // the pair, the odd parts (and R_i of eq. 14) change sign.
        //   G_i even: w_i [S - 3 u.F~ + rho S1 (1.5 |c_i|^2 - 1) + 9 (c_i.u)(c_i.F~)], odd: 3 w_i c_i.F
        //   g_i^eq even: w_i [3 p - 1.5 rho u^2 + 4.5 rho (c_i.u)^2],              odd: 3 w_i rho c_i.u
        //   h_i^eq even: w_i eta mu,                                   odd: 3 w_i c_i.(phi u)
        //   R_i: 3 (1 - 1/(2 tau_h)) w_i c_i.((phi u) - (phi u)_prev)
        const float T0 = S - 3.0f * uFt;
        const float Kax = T0 + 0.5f * rS1, Kdg = T0 + 2.0f * rS1;
        const float Eb = 3.0f * p - 1.5f * rho * u2;
        const float r45 = 4.5f * rho, wr = omega * rho;
        const float hem = ith * emu, ith3 = 3.0f * ith;
        float fs[9], hst[9];
        auto pair = [&](int qa, int qb, float w, float w3, float K, float cu, float cF, float cFt,
                        float cpu, float cd) {
            const float ev = w * (omega * fmaf(r45, cu * cu, Eb) + fgain * fmaf(9.0f * cu, cFt, K));
            const float od = w3 * fmaf(wr, cu, fgain * cF);
            fs[qa] = fmaf(f[qa], om1, ev) + od;
            fs[qb] = fmaf(f[qb], om1, ev) - od;
            const float hev = w * hem;
            const float hod = w * fmaf(ith3, cpu, rcoef * cd);
            hst[qa] = fmaf(h[qa], ith1, hev) + hod;
            hst[qb] = fmaf(h[qb], ith1, hev) - hod;
        };
        pair(1, 3, kWA, k3WA, Kax, ux, Fx, Ftx, phiux, dpx);
        pair(2, 4, kWA, k3WA, Kax, uy, Fy, Fty, phiuy, dpy);
        pair(5, 7, kWD, k3WD, Kdg, ux + uy, Fx + Fy, Ftx + Fty, phiux + phiuy, dpx + dpy);
        pair(6, 8, kWD, k3WD, Kdg, uy - ux, Fy - Fx, Fty - Ftx, phiuy - phiux, dpy - dpx);
        const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
        constexpr bool walls = (BC == 1);
        const int yp = (y + 1 == ny) ? 0 : y + 1, ym = (y == 0) ? ny - 1 : y - 1;
        const bool wall_top = walls && (y == ny - 1), wall_bot = walls && (y == 0);
#pragma unroll
        for (int q = 1; q <= 8; ++q) {
            const int cx = kCX[q], cy = kCY[q];
            // streaming to x + c_i, or back into this node across a wall
            int dx = cx > 0 ? xp : (cx < 0 ? xm : x);
            int dy = cy > 0 ? yp : (cy < 0 ? ym : y);
            int dq = q;
            if ((cy > 0 && wall_top) || (cy < 0 && wall_bot)) {
                dx = x;
                dy = y;
                dq = kOpp[q];
            }
            const unsigned dst = node_off(dy, pitch, dx);
            *pl(fout, P, dq - 1, dst) = fs[q];
            *pl(hout, P, dq, dst) = hst[q];
        }
        // rest population of h: h_0* = h_0 - (h_0 - h_0^eq)/tau_h with h_0 - h_0^eq
        // = -sum_{i!=0} h_i - (w_0 - 1) eta mu; added to the hi/lo pair without rounding h_0
        const float dh0 = (hs + (kW0 - 1.0f) * emu) * ith;
        float nh, e;
        two_sum(h10[0], dh0, nh, e);
        const float nl = h10[kH0Lo] + e;
        float hi2, lo2;
        two_sum(nh, nl, hi2, lo2);
        *pl(hout, P, 0, cell) = hi2;
        *pl(hout, P, kH0Lo, cell) = lo2;
        *pl(pout, P, 0, cell) = p;
        *pl(phiu, P, 0, cell) = phiux;
        *pl(phiu, P, 1, cell) = phiuy;
    }
}

}  // namespace lbpf
