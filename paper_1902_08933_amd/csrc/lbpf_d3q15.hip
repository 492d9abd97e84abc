// Three-dimensional solver of the lbpf library: the phase-field lattice Boltzmann model of
// arXiv:1902.08933, Sec. 3, on the D3Q15 lattice given in Sec. 2.2 (after eq. 25), for gfx950.
//
// The hydrodynamic distribution evolves by eq. (24) with the equilibrium of eq. (33), the force
// distribution of eq. (34) with d = 3, the velocity of eq. (27a) and the pressure of eq. (28)
// (or eq. (29)); the order parameter by eq. (10) with eqs. (11), (14), (18). Stencils are
// eqs. (30a)-(30b) over the fourteen D3Q15 neighbours (six faces, eight corners).
//
// Storage (FP32, SoA planes of nz * ny * pitch floats plus a pad, node (x, y, z) at
// (z * ny + y) * pitch + x): g_1..g_14 (the rest population never enters any output: u uses
// c_0 = 0, eq. (28) sums i != 0), h_0 as an unevaluated pair hi + lo, h_1..h_14, the previous
// pressure and (phi u) in place. 272 bytes of HBM traffic per node and step: 14 + 16 + 1 + 3
// values read and written.
//
// One step is one launch of march3d_kernel. A workgroup owns a TX x TY tile of the x-y plane and
// a chunk of CZ planes, and marches up z one plane per iteration. LDS ring buffers, indexed by
// the global plane number, hold
//   phi (hi, lo) on the tile with a halo of 2, planes z-2 .. z+2 (five slots),
//   mu on the tile with a halo of 1, planes z-1 .. z+1 (three slots),
//   the previous pressure with a halo of 1, planes z-1 .. z+1 (four slots),
// so that each plane's populations are read once for phi, and the node's own populations once
// more (from L2) for the collision. Ring sizes keep every slot written in one iteration distinct
// from the slots any thread may still read from the previous iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbpf.h"
#include "lbpf_cell.hpp"

namespace d3q15 {

using lbpf::pl;
using lbpf::rcp;
using lbpf::two_sum;
using lbpf::wrap;

// D3Q15 in the order of the printed velocity matrix: 0 rest, 1..3 +x +y +z, 4..6 -x -y -z,
// corners 7 (+,+,+), 8 (+,+,-), 9 (+,-,+), 10 (-,+,+), 11..14 their opposites.
__device__ constexpr int kC[15][3] = {{0, 0, 0},   {1, 0, 0},   {0, 1, 0},  {0, 0, 1},  {-1, 0, 0},
                                      {0, -1, 0},  {0, 0, -1},  {1, 1, 1},  {1, 1, -1}, {1, -1, 1},
                                      {-1, 1, 1},  {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
__device__ constexpr int kOpp[15] = {0, 4, 5, 6, 1, 2, 3, 11, 12, 13, 14, 7, 8, 9, 10};
constexpr float kW0 = 2.0f / 9.0f, kWA = 1.0f / 9.0f, kWC = 1.0f / 72.0f;
// 3 w_i in the parts of the collision odd in c_i, which carry the momentum: FP32 values whose
// lattice sum 2 (3 w_A) + 8 (3 w_C) is exactly 1 (the nearest FP32 values of 1/3 and 1/24 sum to
// 1 + 3e-8, which would multiply the momentum by 1 + 3e-8 omega every step).
constexpr float k3WA = 0x1.555556p-2f, k3WC = 0x1.555554p-5f;
static_assert(2.0 * (double)k3WA + 8.0 * (double)k3WC == 1.0, "odd-part weights must sum to 1");

constexpr int kFP = 14;    // g_1..g_14 -> planes 0..13
constexpr int kHP = 16;    // h_0 hi, h_1..h_14, h_0 lo
constexpr int kH0Lo = 15;
// One population copy (the state at one time level): g_1..14 (planes 0..13), h_0 hi, h_1..14,
// h_0 lo (14..29), p (30), (phi u)_x,y,z (31..33). The workspace holds two copies (a step reads
// one and writes the other) and the reduction area; between steps the copy not holding the state
// is free and field evaluation writes its seven planes there. Element (q, x, y, z) of a copy sits
// at q * plane + z * slab + y * pitch + x, with the planes interleaved by grid row (plane =
// pitch3(nx) + 32, pitch = 34 plane) unless the copy would then need per-lane offsets of 2^30
// floats or more, or the environment sets LBPF_STATE_LAYOUT=planar (separate planes).
constexpr int kCopyG = 0, kCopyH = 14, kCopyP = 30, kCopyPhiU = 31, kCopyPlanes = 34;
constexpr int kNumFields = 7;
constexpr long kPlanePad = 4160;
constexpr int kRedBlocks = 2048, kRedSlots = 4;
constexpr size_t kRedDoubles = (size_t)kRedBlocks * kRedSlots + 64;

struct Model3 {
    int nx, ny, nz;
    int pitch;             // floats between rows (y) of a copy
    int slab;              // ny * pitch: floats between z planes of the grid
    long long plane;       // floats between planes (q) of a copy
    long long copy;        // floats per population copy (34 planes and a pad)
    int variant, pscheme, fsurf, visc, bc, clamp;
    float beta4, kappa, eta, gammaM, rhoA, rhoB, drho, inv_nuA, inv_nuB, muA, muB;
    float inv_tau_h, src_coef, fx, fy, fz, grav;
    double d_rhoA, d_rhoB, d_beta, d_kappa;
};

// offset of node (x, y, z) in a plane: z * slab needs the full 32-bit product (a slab may hold
// 2^24 floats or more), y * pitch fits the 24-bit multiplier (both sides < 2^24)
__device__ __forceinline__ unsigned node3(const Model3& m, int z, int y, int x) {
    return (unsigned)z * (unsigned)m.slab + (unsigned)__umul24(y, m.pitch) + (unsigned)x;
}

// plane read for a stencil ghost: periodic wrap (BC 0) or the mirror image about a wall half a
// cell outside the first / last fluid plane (BC 1), clamped for planes no active node reads
template <int BC>
__device__ __forceinline__ int src_z(int z, int nz) {
    if (BC == 0) return wrap(z, nz);
    if (z < 0) z = -1 - z;
    else if (z >= nz) z = 2 * nz - 1 - z;
    return z < 0 ? 0 : (z >= nz ? nz - 1 : z);
}

// mirror plane of a stencil ghost beyond a wall (the plane whose values the ghost takes)
template <int BC>
__device__ __forceinline__ int mirror_z(int z, int nz) {
    if (BC == 0) return z;
    if (z < 0) return -1 - z;
    if (z >= nz) return 2 * nz - 1 - z;
    return z;
}

template <int TX, int TY, int PF>
struct Lds3 {
    static constexpr int PX = TX + 4, PN = PX * (TY + 4);  // phi planes, halo 2
    static constexpr int MX = TX + 2, MN = MX * (TY + 2);  // mu and pressure planes, halo 1
    static constexpr int RP = 5, RM = 3, RQ = 4;
    float phh[RP * PN];
    float phl[RP * PN];
    float mu[RM * MN];
    float p[RQ * MN];
    // PF: the owned node's sixteen h values of the next two planes, [slot][q][thread] (each
    // thread reads back only what it wrote, so the stash needs no barrier)
    float own[PF ? 2 * kHP * TX * TY : 1];
};

// phi = sum_i h_i (eq. 18) as an FP32 pair from the sixteen stored h values of a node
__device__ __forceinline__ void phi_pair16(const float (&h)[kHP], float& hi, float& lo) {
    float s = 0.0f;
#pragma unroll
    for (int q = 1; q <= 14; ++q) s += h[q];
    float e;
    two_sum(h[0], s, hi, e);
    lo = h[kH0Lo] + e;
}

// offset of the (possibly ghost) node (x, y, z): x, y wrapped, z wrapped or mirrored
template <int BC>
__device__ __forceinline__ unsigned src_node(const Model3& m, int x, int y, int z) {
    return node3(m, src_z<BC>(z, m.nz), wrap(y, m.ny), wrap(x, m.nx));
}

template <int BC>
__device__ __forceinline__ void phi_at(const Model3& m, const float* __restrict__ hin, int x, int y,
                                       int z, float& hi, float& lo) {
    const unsigned c = src_node<BC>(m, x, y, z);
    float h[kHP];
#pragma unroll
    for (int q = 0; q < kHP; ++q) h[q] = *pl(hin, m.plane, q, c);
    phi_pair16(h, hi, lo);
}

// eq. (8) with the Laplacian of eq. (30b) over the D3Q15 neighbours, on differences of phi
// pairs; bm, bc, bp are the LDS bases of the planes below, at and above, (px, py) the column
// in phi-plane coordinates. Laplacian: 2/3 sum_faces (z_f - z) + 1/12 sum_corners (z_c - z).
template <int PX>
__device__ __forceinline__ float mu_at3(const Model3& m, const float* phh, const float* phl, int bm,
                                        int bc, int bp, int px, int py) {
    const int o = py * PX + px, c = bc + o;
    const float ch = phh[c], cl = phl[c];
    auto d = [&](int i) { return (phh[i] - ch) + (phl[i] - cl); };
    const float faces = ((d(c + 1) + d(c - 1)) + (d(c + PX) + d(c - PX))) + (d(bm + o) + d(bp + o));
    const float cm = (d(bm + o + PX + 1) + d(bm + o + PX - 1)) + (d(bm + o - PX + 1) + d(bm + o - PX - 1));
    const float cp = (d(bp + o + PX + 1) + d(bp + o + PX - 1)) + (d(bp + o - PX + 1) + d(bp + o - PX - 1));
    const float lap = (2.0f / 3.0f) * faces + (1.0f / 12.0f) * (cm + cp);
    const float a = ch + cl, b = (ch - 1.0f) + cl, cc = (ch - 0.5f) + cl;
    return m.beta4 * a * b * cc - m.kappa * lap;
}

struct Stencil3 {
    float phh, phl;
    float gphi[3];
    float mu, gmu[3], lapmu;
    float gp[3];
};

// eq. (30a) over the D3Q15 neighbours: grad_x z = (z_E - z_W)/3 + 1/24 sum over the four
// corner pairs (z(x+1, y+sy, z+sz) - z(x-1, y+sy, z+sz)), and cyclically.
template <class Dz>
__device__ __forceinline__ void grad3(Dz dz, int bm, int bc, int bp, int o, int RX, float* g) {
    // dz(a, b) = z[a] - z[b]
    const int E = 1, N = RX;
    g[0] = (1.0f / 3.0f) * dz(bc + o + E, bc + o - E)
         + (1.0f / 24.0f) * ((dz(bm + o + N + E, bm + o + N - E) + dz(bm + o - N + E, bm + o - N - E))
                           + (dz(bp + o + N + E, bp + o + N - E) + dz(bp + o - N + E, bp + o - N - E)));
    g[1] = (1.0f / 3.0f) * dz(bc + o + N, bc + o - N)
         + (1.0f / 24.0f) * ((dz(bm + o + N + E, bm + o - N + E) + dz(bm + o + N - E, bm + o - N - E))
                           + (dz(bp + o + N + E, bp + o - N + E) + dz(bp + o + N - E, bp + o - N - E)));
    g[2] = (1.0f / 3.0f) * dz(bp + o, bm + o)
         + (1.0f / 24.0f) * ((dz(bp + o + N + E, bm + o + N + E) + dz(bp + o + N - E, bm + o + N - E))
                           + (dz(bp + o - N + E, bm + o - N + E) + dz(bp + o - N - E, bm + o - N - E)));
}

template <class L>
__device__ __forceinline__ Stencil3 gather3(const L& S, int pm, int pc, int pp, int mm, int mc,
                                            int mp, int qm, int qc, int qp, int tx, int ty) {
    Stencil3 s;
    const int po = (ty + 2) * L::PX + tx + 2, mo = (ty + 1) * L::MX + tx + 1;
    s.phh = S.phh[pc + po];
    s.phl = S.phl[pc + po];
    grad3([&](int a, int b) { return (S.phh[a] - S.phh[b]) + (S.phl[a] - S.phl[b]); }, pm, pc, pp, po,
          L::PX, s.gphi);
    grad3([&](int a, int b) { return S.mu[a] - S.mu[b]; }, mm, mc, mp, mo, L::MX, s.gmu);
    grad3([&](int a, int b) { return S.p[a] - S.p[b]; }, qm, qc, qp, mo, L::MX, s.gp);
    const float* z = S.mu;
    const int c = mc + mo, N = L::MX;
    const float mu = z[c];
    s.mu = mu;
    auto d = [&](int i) { return z[i] - mu; };
    const float faces = ((d(c + 1) + d(c - 1)) + (d(c + N) + d(c - N))) + (d(mm + mo) + d(mp + mo));
    const float cm = (d(mm + mo + N + 1) + d(mm + mo + N - 1)) + (d(mm + mo - N + 1) + d(mm + mo - N - 1));
    const float cp = (d(mp + mo + N + 1) + d(mp + mo + N - 1)) + (d(mp + mo - N + 1) + d(mp + mo - N - 1));
    s.lapmu = (2.0f / 3.0f) * faces + (1.0f / 12.0f) * (cm + cp);
    return s;
}

// One node: closure, force, velocity (eq. 27a), source, F~, pressure (eq. 28 / 29) and, when
// colliding, both BGK collisions with push streaming. g holds g_1..g_14, h the sixteen h planes.
template <bool COLLIDE, int BC>
__device__ __forceinline__ void cell3(const Model3& m, int x, int y, int z, unsigned cell,
                                      const float (&g14)[kFP], const float (&h16)[kHP],
                                      const float (&pu)[3], const Stencil3& st,
                                      float* __restrict__ gout, float* __restrict__ hout,
                                      float* __restrict__ pout, float* __restrict__ phiu,
                                      float* __restrict__ fields) {
    const long long P = m.plane;
    float g[15];
#pragma unroll
    for (int q = 1; q <= 14; ++q) g[q] = g14[q - 1];
    const float phi = st.phh + st.phl;
    const float phic = m.clamp ? fminf(fmaxf(phi, 0.0f), 1.0f) : phi;
    const float rho = m.rhoB + m.drho * phic;
    float F[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = (m.fsurf == 0) ? st.mu * st.gphi[a] : -phi * st.gmu[a];
    F[0] += m.fx;
    F[1] += m.fy;
    F[2] += m.fz - (rho - m.rhoA) * m.grav;
    // eq. (27a): u = (sum_i c_i g_i + F/2) / rho; corners 7..10 and their opposites 11..14
    const float c7 = g[7] - g[11], c8 = g[8] - g[12], c9 = g[9] - g[13], c10 = g[10] - g[14];
    const float mx = (g[1] - g[4]) + ((c7 + c8) + (c9 - c10));
    const float my = (g[2] - g[5]) + ((c7 + c8) + (c10 - c9));
    const float mz = (g[3] - g[6]) + ((c7 - c8) + (c9 + c10));
    const float irho = rcp(rho);
    const float u[3] = {(mx + 0.5f * F[0]) * irho, (my + 0.5f * F[1]) * irho, (mz + 0.5f * F[2]) * irho};
    const float S1 = (m.variant == 0) ? -m.gammaM * st.lapmu : 0.0f;
    const float gr[3] = {m.drho * st.gphi[0], m.drho * st.gphi[1], m.drho * st.gphi[2]};
    const float rS1 = rho * S1;
    const float S = ((u[0] * gr[0] + u[1] * gr[1]) + u[2] * gr[2]) + rS1;
    float Ft[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Ft[a] = F[a] - st.gp[a] + (1.0f / 3.0f) * gr[a];
    const float uFt = (u[0] * Ft[0] + u[1] * Ft[1]) + u[2] * Ft[2];
    float nu;
    if (m.visc == 0) nu = rcp(phic * (m.inv_nuA - m.inv_nuB) + m.inv_nuB);
    else nu = ((phi >= 0.5f) ? m.muA : m.muB) * irho;
    const float tau_g = 3.0f * nu + 0.5f;
    // eq. (28): p = c_s^2/(1 - w_0) [sum_{i!=0} g_i + S/2 + rho s_0(u) + (tau_g - 1/2) G_0] with
    // c_s^2/(1 - w_0) = 3/7 and rho s_0(u) = -rho |u|^2 / 3
    const float u2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    float sumg = 0.0f;
#pragma unroll
    for (int q = 1; q <= 14; ++q) sumg += g[q];
    float bracket = sumg + 0.5f * S - (1.0f / 3.0f) * rho * u2;
    if (m.pscheme == 0) {
        // eq. (34) at i = 0: G_0 = w_0 (S - u.F~/c_s^2 - rho S1)
        bracket += (tau_g - 0.5f) * (kW0 * (S - 3.0f * uFt - rS1));
    } else if (m.pscheme == 1) {
        const float uFp = (u[0] * (F[0] - st.gp[0]) + u[1] * (F[1] - st.gp[1])) + u[2] * (F[2] - st.gp[2]);
        bracket += (tau_g - 0.5f) * (kW0 * ((2.0f / 3.0f) * rS1 - 3.0f * uFp));
    }
    const float p = (3.0f / 7.0f) * bracket;
    const float pu_new[3] = {phi * u[0], phi * u[1], phi * u[2]};

    if constexpr (!COLLIDE) {
        *pl(fields, P, 0, cell) = phi;
        *pl(fields, P, 1, cell) = rho;
        *pl(fields, P, 2, cell) = u[0];
        *pl(fields, P, 3, cell) = u[1];
        *pl(fields, P, 4, cell) = u[2];
        *pl(fields, P, 5, cell) = p;
        *pl(fields, P, 6, cell) = st.mu;
    } else {
        const float omega = rcp(tau_g), om1 = 1.0f - omega, fgain = 1.0f - 0.5f * omega;
        const float emu = m.eta * st.mu;
        const float dpu[3] = {pu_new[0] - pu[0], pu_new[1] - pu[1], pu_new[2] - pu[2]};
        const float rcoef = 3.0f * m.src_coef;
        const float ith = m.inv_tau_h, ith1 = 1.0f - ith;
        // Collisions by pairs of opposite directions; with d = 3 and c_s^2 = 1/3, eq. (34) is
        //   G_i = w_i [S - 3 u.F~ + rho S1 (|c_i|^2 - 1) + 9 (c_i.u)(c_i.F~) + 3 c_i.F],
        // eq. (33) for i != 0 is g_i^eq = w_i [3 p - 1.5 rho u^2 + 4.5 rho (c_i.u)^2 + 3 rho c_i.u],
        // eq. (11) h_i^eq = w_i [eta mu + 3 c_i.(phi u)], eq. (14) R_i = 3 (1 - 1/(2 tau_h))
        // w_i c_i.d(phi u); the parts even in c_i are shared by the pair, odd parts change sign.
        const float T0 = S - 3.0f * uFt;
        const float Kf = T0, Kc = T0 + 2.0f * rS1;  // |c|^2 = 1 (faces), 3 (corners)
        const float Eb = 3.0f * p - 1.5f * rho * u2;
        const float r45 = 4.5f * rho, wr = omega * rho;
        const float hem = ith * emu, ith3 = 3.0f * ith;
        float gs[15], hs[15];
        float hsum = 0.0f;
#pragma unroll
        for (int q = 1; q <= 14; ++q) hsum += h16[q];
        auto pair = [&](int qa, int qb, float w, float w3, float K, float cu, float cF, float cFt,
                        float cpu, float cd) {
            const float ev = w * (omega * fmaf(r45, cu * cu, Eb) + fgain * fmaf(9.0f * cu, cFt, K));
            const float od = w3 * fmaf(wr, cu, fgain * cF);
            gs[qa] = fmaf(g[qa], om1, ev) + od;
            gs[qb] = fmaf(g[qb], om1, ev) - od;
            const float hev = w * hem;
            const float hod = w * fmaf(ith3, cpu, rcoef * cd);
            hs[qa] = fmaf(h16[qa], ith1, hev) + hod;
            hs[qb] = fmaf(h16[qb], ith1, hev) - hod;
        };
#pragma unroll
        for (int a = 0; a < 3; ++a) pair(1 + a, 4 + a, kWA, k3WA, Kf, u[a], F[a], Ft[a], pu_new[a], dpu[a]);
        auto dot = [](float sx, float sy, float sz, const float* v) { return (sx * v[0] + sy * v[1]) + sz * v[2]; };
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int qa = 7 + k, qb = 11 + k;
            const float sx = (float)kC[qa][0], sy = (float)kC[qa][1], sz = (float)kC[qa][2];
            pair(qa, qb, kWC, k3WC, Kc, dot(sx, sy, sz, u), dot(sx, sy, sz, F), dot(sx, sy, sz, Ft),
                 dot(sx, sy, sz, pu_new), dot(sx, sy, sz, dpu));
        }
        const int nx = m.nx, ny = m.ny, nz = m.nz;
        const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
        const int yp = (y + 1 == ny) ? 0 : y + 1, ym = (y == 0) ? ny - 1 : y - 1;
        const int zp = (z + 1 == nz) ? 0 : z + 1, zm = (z == 0) ? nz - 1 : z - 1;
        constexpr bool walls = (BC == 1);
        const bool wall_top = walls && (z == nz - 1), wall_bot = walls && (z == 0);
#pragma unroll
        for (int q = 1; q <= 14; ++q) {
            const int cx = kC[q][0], cy = kC[q][1], cz = kC[q][2];
            int dx = cx > 0 ? xp : (cx < 0 ? xm : x);
            int dy = cy > 0 ? yp : (cy < 0 ? ym : y);
            int dz = cz > 0 ? zp : (cz < 0 ? zm : z);
            int dq = q;
            if ((cz > 0 && wall_top) || (cz < 0 && wall_bot)) {
                dx = x;
                dy = y;
                dz = z;
                dq = kOpp[q];
            }
            const unsigned dst = node3(m, dz, dy, dx);
            *pl(gout, P, dq - 1, dst) = gs[q];
            *pl(hout, P, dq, dst) = hs[q];
        }
        // h_0* = h_0 + (sum_{i!=0} h_i + (w_0 - 1) eta mu) / tau_h, added to the pair unrounded
        const float dh0 = (hsum + (kW0 - 1.0f) * emu) * ith;
        float nh, e;
        two_sum(h16[0], dh0, nh, e);
        const float nl = h16[kH0Lo] + e;
        float hi2, lo2;
        two_sum(nh, nl, hi2, lo2);
        *pl(hout, P, 0, cell) = hi2;
        *pl(hout, P, kH0Lo, cell) = lo2;
        *pl(pout, P, 0, cell) = p;
#pragma unroll
        for (int a = 0; a < 3; ++a) *pl(phiu, P, a, cell) = pu_new[a];
    }
}

// XCD-aware order: block b runs on XCD b % 8; each XCD takes a contiguous range of tiles
__device__ __forceinline__ int xcd_order(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, loc = b / 8;
    return xcd * per + (xcd < rem ? xcd : rem) + loc;
}

// PF = 1 software-pipelines the loads: the next phi plane's populations (each thread loads its
// own column's node and at most NHK halo nodes) and the next pressure plane are loaded into
// registers before the current plane's update, so that their latency overlaps the collision
// arithmetic; the owned node's h values, needed again two planes later for its collision, are
// kept in a thread-private LDS stash instead of being read a second time. The arithmetic is the
// same for PF = 0 and 1.
template <int TX, int TY, bool COLLIDE, int BC, int PF>
__global__ __launch_bounds__(TX * TY) void march3d_kernel(Model3 m, const float* __restrict__ gin,
                                                          float* __restrict__ gout,
                                                          const float* __restrict__ hin,
                                                          float* __restrict__ hout,
                                                          const float* __restrict__ pin,
                                                          float* __restrict__ pout,
                                                          const float* __restrict__ phiu_in,
                                                          float* __restrict__ phiu_out,
                                                          float* __restrict__ fields, int ntx,
                                                          int nty, int cz) {
    using L = Lds3<TX, TY, PF>;
    constexpr int NT = TX * TY, PX = L::PX, PN = L::PN, MX = L::MX, MN = L::MN;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    L& S = *reinterpret_cast<L*>(lds_raw);
    const int nblk = gridDim.x;
    const int blk = xcd_order(blockIdx.x, nblk);
    const int tile = blk % (ntx * nty), chunk = blk / (ntx * nty);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int zs = chunk * cz, ze = min(zs + cz, m.nz);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const long long P = m.plane;
    auto pslot = [](int z) { return ((z + 10) % 5) * PN; };
    auto mslot = [](int z) { return ((z + 3) % 3) * MN; };
    auto qslot = [](int z) { return ((z + 4) % 4) * MN; };

    auto publish_phi = [&](int z) {
        const int b = pslot(z);
        for (int j = tid; j < PN; j += NT) {
            float hi, lo;
            phi_at<BC>(m, hin, x0 + j % PX - 2, y0 + j / PX - 2, z, hi, lo);
            S.phh[b + j] = hi;
            S.phl[b + j] = lo;
        }
    };
    auto publish_p = [&](int z) {
        const int b = qslot(z);
        const int sz = src_z<BC>(z, m.nz);
        for (int j = tid; j < MN; j += NT)
            S.p[b + j] = *pl(pin, P, 0, node3(m, sz, wrap(y0 + j / MX - 1, m.ny), wrap(x0 + j % MX - 1, m.nx)));
    };
    // mu on plane z (global index, possibly a ghost beyond a wall: then the mirror plane's mu,
    // computed from the phi planes around the mirror plane, which the ring also holds)
    auto compute_mu = [&](int z) {
        const int c = mirror_z<BC>(z, m.nz);
        const int bm = pslot(c - 1), bc = pslot(c), bp = pslot(c + 1), b = mslot(z);
        for (int j = tid; j < MN; j += NT)
            S.mu[b + j] = mu_at3<PX>(m, S.phh, S.phl, bm, bc, bp, j % MX + 1, j / MX + 1);
    };

    // PF: the halo of a phi plane (PN - NT nodes: rows 0, 1, TY+2, TY+3 at full width, then
    // columns 0, 1, TX+2, TX+3 of rows 2 .. TY+1) spread over the threads, NHK per thread
    constexpr int NHALO = PN - NT, NHK = (NHALO + NT - 1) / NT, NPP = (MN + NT - 1) / NT;
    auto halo_pos = [](int k, int& lx, int& ly) {
        if (k < 4 * PX) {
            const int r = k / PX;
            ly = r < 2 ? r : TY + r;
            lx = k % PX;
        } else {
            const int k2 = k - 4 * PX, c4 = k2 % 4;
            ly = 2 + k2 / 4;
            lx = c4 < 2 ? c4 : TX + c4;
        }
    };
    float hin_own[PF ? kHP : 1];
    float hq[PF ? NHK : 1][kHP];
    float pq[PF ? NPP : 1];
    auto load_halo = [&](int zf, int zp) {
        if constexpr (PF != 0) {
            const unsigned c0 = src_node<BC>(m, x0 + tx, y0 + ty, zf);
#pragma unroll
            for (int q = 0; q < kHP; ++q) hin_own[q] = *pl(hin, P, q, c0);
#pragma unroll
            for (int k = 0; k < NHK; ++k) {
                const int j = tid + k * NT;
                if (j < NHALO) {
                    int lx, ly;
                    halo_pos(j, lx, ly);
                    const unsigned c = src_node<BC>(m, x0 + lx - 2, y0 + ly - 2, zf);
#pragma unroll
                    for (int q = 0; q < kHP; ++q) hq[k][q] = *pl(hin, P, q, c);
                }
            }
#pragma unroll
            for (int k = 0; k < NPP; ++k) {
                const int j = tid + k * NT;
                if (j < MN) pq[k] = *pl(pin, P, 0, src_node<BC>(m, x0 + j % MX - 1, y0 + j / MX - 1, zp));
            }
        }
    };
    auto store_halo = [&](int zf, int zp) {
        if constexpr (PF != 0) {
            const int b = pslot(zf), bq = qslot(zp);
            const int o = b + (ty + 2) * PX + tx + 2;
            phi_pair16(hin_own, S.phh[o], S.phl[o]);
            float* st = S.own + (zf & 1) * (kHP * NT) + tid;
#pragma unroll
            for (int q = 0; q < kHP; ++q) st[q * NT] = hin_own[q];
#pragma unroll
            for (int k = 0; k < NHK; ++k) {
                const int j = tid + k * NT;
                if (j < NHALO) {
                    int lx, ly;
                    halo_pos(j, lx, ly);
                    phi_pair16(hq[k], S.phh[b + ly * PX + lx], S.phl[b + ly * PX + lx]);
                }
            }
#pragma unroll
            for (int k = 0; k < NPP; ++k) {
                const int j = tid + k * NT;
                if (j < MN) S.p[bq + j] = pq[k];
            }
        }
    };

    // prologue: phi planes zs-2 .. zs+1, pressure planes zs-1, zs, mu planes zs-1, zs (with PF,
    // planes zs and zs+1 through the stash path, and the first iteration's loads in flight)
    if (PF) {
        publish_phi(zs - 2);
        publish_phi(zs - 1);
        load_halo(zs, zs - 1);
        store_halo(zs, zs - 1);
        load_halo(zs + 1, zs);
        store_halo(zs + 1, zs);
        load_halo(zs + 2, zs + 1);
    } else {
        for (int z = zs - 2; z <= zs + 1; ++z) publish_phi(z);
        publish_p(zs - 1);
        publish_p(zs);
    }
    __syncthreads();
    compute_mu(zs - 1);
    compute_mu(zs);

    const int x = x0 + tx, y = y0 + ty;
    const bool col_active = x < m.nx && y < m.ny;
    // PF: the owned node's g and (phi u) of the next plane are loaded with the halo prefetch
    float gn[PF ? kFP : 1], pun[PF ? 3 : 1];
    auto load_own = [&](int zz) {
        if constexpr (PF != 0) {
            const unsigned c = node3(m, zz, y, x);
#pragma unroll
            for (int q = 0; q < kFP; ++q) gn[q] = *pl(gin, P, q, c);
#pragma unroll
            for (int a = 0; a < 3; ++a) pun[a] = *pl(phiu_in, P, a, c);
        }
    };
    if (PF && col_active) load_own(zs);
    for (int z = zs; z < ze; ++z) {
        float g[kFP], h[kHP], pu[3];
        unsigned cell = 0;
        if (col_active) {
            cell = node3(m, z, y, x);
            if (PF) {
#pragma unroll
                for (int q = 0; q < kFP; ++q) g[q] = gn[PF ? q : 0];
#pragma unroll
                for (int a = 0; a < 3; ++a) pu[a] = pun[PF ? a : 0];
            } else {
#pragma unroll
                for (int q = 0; q < kFP; ++q) g[q] = *pl(gin, P, q, cell);
#pragma unroll
                for (int a = 0; a < 3; ++a) pu[a] = *pl(phiu_in, P, a, cell);
            }
        }
        if (PF) {
            // the owned node's h from the stash (written two iterations ago by this thread),
            // read before this iteration's store reuses the slot
            const float* st = S.own + (z & 1) * (kHP * NT) + tid;
#pragma unroll
            for (int q = 0; q < kHP; ++q) h[q] = st[q * NT];
            store_halo(z + 2, z + 1);
        } else {
            if (col_active) {
#pragma unroll
                for (int q = 0; q < kHP; ++q) h[q] = *pl(hin, P, q, cell);
            }
            publish_phi(z + 2);
            publish_p(z + 1);
        }
        __syncthreads();
        compute_mu(z + 1);
        __syncthreads();
        if (PF && z + 1 < ze) {
            load_halo(z + 3, z + 2);
            if (col_active) load_own(z + 1);
        }
        if (col_active) {
            const Stencil3 st = gather3(S, pslot(z - 1), pslot(z), pslot(z + 1), mslot(z - 1), mslot(z),
                                        mslot(z + 1), qslot(z - 1), qslot(z), qslot(z + 1), tx, ty);
            cell3<COLLIDE, BC>(m, x, y, z, cell, g, h, pu, st, gout, hout, pout, phiu_out, fields);
        }
    }
}

// ---- initial state: equilibria of eq. (11) and eq. (33) at (phi0, mu0, u0, p0) --------------
template <int BC>
__global__ void init3d_kernel(Model3 m, const float* __restrict__ phi0, const float* __restrict__ ux0,
                              const float* __restrict__ uy0, const float* __restrict__ uz0,
                              const float* __restrict__ p0, float* __restrict__ g,
                              float* __restrict__ h, float* __restrict__ pp, float* __restrict__ phiu) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= m.nx) return;
    const int nx = m.nx, ny = m.ny;
    auto at = [&](int dx, int dy, int dz) {
        const long long k = ((long long)src_z<BC>(z + dz, m.nz) * ny + wrap(y + dy, ny)) * nx + wrap(x + dx, nx);
        return phi0[k];
    };
    const float c = at(0, 0, 0);
    const float faces = ((at(1, 0, 0) - c) + (at(-1, 0, 0) - c)) + ((at(0, 1, 0) - c) + (at(0, -1, 0) - c))
                      + ((at(0, 0, 1) - c) + (at(0, 0, -1) - c));
    float corners = 0.0f;
    for (int sz = -1; sz <= 1; sz += 2)
        for (int sy = -1; sy <= 1; sy += 2)
            corners += (at(1, sy, sz) - c) + (at(-1, sy, sz) - c);
    const float lap = (2.0f / 3.0f) * faces + (1.0f / 12.0f) * corners;
    const float mu = m.beta4 * c * (c - 1.0f) * (c - 0.5f) - m.kappa * lap;
    const long long in = ((long long)z * ny + y) * nx + x;
    const float u[3] = {ux0 ? ux0[in] : 0.0f, uy0 ? uy0[in] : 0.0f, uz0 ? uz0[in] : 0.0f};
    const float p = p0 ? p0[in] : 0.0f;
    const float phic = m.clamp ? fminf(fmaxf(c, 0.0f), 1.0f) : c;
    const float rho = m.rhoB + m.drho * phic;
    const unsigned cell = node3(m, z, y, x);
    const long long P = m.plane;
    const float emu = m.eta * mu, u2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    const float pu[3] = {c * u[0], c * u[1], c * u[2]};
    float hi, lo;
    two_sum(c, (kW0 - 1.0f) * emu, hi, lo);
    *pl(h, P, 0, cell) = hi;
    *pl(h, P, kH0Lo, cell) = lo;
#pragma unroll
    for (int q = 1; q <= 14; ++q) {
        const float w = q <= 6 ? kWA : kWC;
        const float cu = (kC[q][0] * u[0] + kC[q][1] * u[1]) + kC[q][2] * u[2];
        const float cp = (kC[q][0] * pu[0] + kC[q][1] * pu[1]) + kC[q][2] * pu[2];
        *pl(g, P, q - 1, cell) = w * (3.0f * p + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2));
        *pl(h, P, q, cell) = w * (emu + 3.0f * cp);
    }
    *pl(pp, P, 0, cell) = p;
#pragma unroll
    for (int a = 0; a < 3; ++a) *pl(phiu, P, a, cell) = pu[a];
}

// ---- FP64 diagnostics: deterministic two-pass reductions --------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh, bool is_max) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o);
        v = is_max ? fmax(v, w) : v + w;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = sh[0];
        for (int i = 1; i < 4; ++i) r = is_max ? fmax(r, sh[i]) : r + sh[i];
    }
    return r;
}

// per-block partials of sum phi (FP64 sum of the stored h), sum rho, max |u| (from the field
// scratch), non-finite stored values
__global__ __launch_bounds__(256) void diag3d_partial_kernel(Model3 m, const float* __restrict__ g,
                                                             const float* __restrict__ h,
                                                             const float* __restrict__ pp,
                                                             const float* __restrict__ phiu,
                                                             const float* __restrict__ fields,
                                                             double* __restrict__ part) {
    __shared__ double sh[4];
    const long long n = (long long)m.nx * m.ny * m.nz, P = m.plane;
    double sphi = 0.0, srho = 0.0, umax = 0.0, bad = 0.0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % m.nx);
        const long long r = k / m.nx;
        const int y = (int)(r % m.ny), z = (int)(r / m.ny);
        const unsigned cell = node3(m, z, y, x);
        double phi = (double)*pl(h, P, 0, cell) + (double)*pl(h, P, kH0Lo, cell);
        for (int q = 1; q <= 14; ++q) phi += (double)*pl(h, P, q, cell);
        double phc = phi;
        if (m.clamp) phc = phc < 0.0 ? 0.0 : (phc > 1.0 ? 1.0 : phc);
        sphi += phi;
        srho += m.d_rhoB + (m.d_rhoA - m.d_rhoB) * phc;
        const double ux = *pl(fields, P, 2, cell), uy = *pl(fields, P, 3, cell), uz = *pl(fields, P, 4, cell);
        const double um = sqrt(ux * ux + uy * uy + uz * uz);
        umax = (um > umax || um != um) ? um : umax;
        int nb = 0;
        for (int q = 0; q < kFP; ++q) nb += !isfinite(*pl(g, P, q, cell));
        for (int q = 0; q < kHP; ++q) nb += !isfinite(*pl(h, P, q, cell));
        nb += !isfinite(*pl(pp, P, 0, cell));
        for (int a = 0; a < 3; ++a) nb += !isfinite(*pl(phiu, P, a, cell));
        bad += nb;
    }
    const double a = block_sum(sphi, sh, false);
    const double b = block_sum(srho, sh, false);
    const double c = block_sum(umax, sh, true);
    const double d = block_sum(bad, sh, false);
    if (threadIdx.x == 0) {
        double* o = part + (size_t)blockIdx.x * kRedSlots;
        o[0] = a; o[1] = b; o[2] = c; o[3] = d;
    }
}

// second pass: slot s of every partial reduced in a fixed order; bit s of maxmask takes the
// maximum instead of the sum
__global__ __launch_bounds__(256) void reduce3d_final_kernel(const double* __restrict__ part, int nblk,
                                                             unsigned maxmask, double* __restrict__ out) {
    __shared__ double sh[4];
    for (int s = 0; s < kRedSlots; ++s) {
        const bool is_max = (maxmask >> s) & 1u;
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) {
            const double w = part[(size_t)b * kRedSlots + s];
            v = is_max ? ((w > v || w != w) ? w : v) : v + w;
        }
        const double r = block_sum(v, sh, is_max);
        if (threadIdx.x == 0) out[s] = r;
    }
}

// phi in FP64 of the (possibly ghost) node (x, y, z): h_0 hi + h_0 lo + sum_{i!=0} h_i (eq. 18)
template <int BC>
__device__ __forceinline__ double phi64_at(const Model3& m, const float* __restrict__ h, int x, int y, int z) {
    const unsigned c = src_node<BC>(m, x, y, z);
    double phi = (double)*pl(h, m.plane, 0, c) + (double)*pl(h, m.plane, kH0Lo, c);
    for (int q = 1; q <= 14; ++q) phi += (double)*pl(h, m.plane, q, c);
    return phi;
}

// Laplace pressure of Sec. 4.2 in FP64, P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p
// with p0 = phi psi' - psi, psi = beta phi^2 (phi - 1)^2, eqs. (30a)-(30b) over the D3Q15
// neighbours on FP64 phi; per-block sums of P and counts over r <= r_in and r >= r_out from
// (xc, yc, zc), distances periodic in x, y (and z when periodic)
template <int BC>
__global__ __launch_bounds__(256) void laplace3d_partial_kernel(Model3 m, const float* __restrict__ h,
                                                                const float* __restrict__ fields,
                                                                double xc, double yc, double zc,
                                                                double r_in, double r_out,
                                                                double* __restrict__ part) {
    __shared__ double sh[4];
    const long long n = (long long)m.nx * m.ny * m.nz;
    double s_in = 0.0, c_in = 0.0, s_out = 0.0, c_out = 0.0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % m.nx);
        const long long r = k / m.nx;
        const int y = (int)(r % m.ny), z = (int)(r / m.ny);
        const double c = phi64_at<BC>(m, h, x, y, z);
        double g[3] = {0.0, 0.0, 0.0}, lap = 0.0;
        for (int i = 1; i < 15; ++i) {
            const double w = i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0;
            const double v = phi64_at<BC>(m, h, x + kC[i][0], y + kC[i][1], z + kC[i][2]);
            for (int a = 0; a < 3; ++a) g[a] += 3.0 * w * kC[i][a] * v;
            lap += 6.0 * w * (v - c);
        }
        const double psi = m.d_beta * c * c * (c - 1.0) * (c - 1.0);
        const double dpsi = 4.0 * m.d_beta * c * (c - 1.0) * (c - 0.5);
        const double p = (double)*pl(fields, m.plane, 5, node3(m, z, y, x));
        const double Pt = (c * dpsi - psi) - m.d_kappa * c * lap
                        + 0.5 * m.d_kappa * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + p;
        double dx = fabs(x - xc), dy = fabs(y - yc), dz = fabs(z - zc);
        dx = fmin(dx, m.nx - dx);
        dy = fmin(dy, m.ny - dy);
        if (BC == 0) dz = fmin(dz, m.nz - dz);
        const double rr = sqrt(dx * dx + dy * dy + dz * dz);
        if (rr <= r_in) { s_in += Pt; c_in += 1.0; }
        if (rr >= r_out) { s_out += Pt; c_out += 1.0; }
    }
    const double a = block_sum(s_in, sh, false);
    const double b = block_sum(c_in, sh, false);
    const double cc = block_sum(s_out, sh, false);
    const double d = block_sum(c_out, sh, false);
    if (threadIdx.x == 0) {
        double* o = part + (size_t)blockIdx.x * kRedSlots;
        o[0] = a; o[1] = b; o[2] = cc; o[3] = d;
    }
}

// one field plane (padded layout) into a dense [nz][ny][nx] array
__global__ void compact3d_kernel(Model3 m, const float* __restrict__ src, float* __restrict__ dst) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= m.nx) return;
    dst[((long long)z * m.ny + y) * m.nx + x] = *pl(src, m.plane, 0, node3(m, z, y, x));
}

// ---- launch shapes -------------------------------------------------------------------------
struct Shape3 { int tx, ty, cz, pf; };
static const Shape3 kShapes3[] = {{32, 8, 32, 0},  {32, 8, 64, 0},  {64, 4, 32, 0}, {64, 8, 32, 0},
                                  {32, 16, 32, 0}, {64, 8, 64, 0},  {32, 8, 16, 0}, {64, 4, 64, 0},
                                  {32, 8, 32, 1},  {32, 8, 16, 1},  {64, 4, 32, 1}, {64, 8, 32, 1},
                                  {32, 16, 32, 1}, {64, 8, 16, 1},  {64, 4, 16, 1}, {32, 8, 8, 1}};
constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);
constexpr int kDefaultShape3 = 0;

template <int TX, int TY, bool C, int BC, int PF>
static hipError_t launch_t(const Model3& m, int cz, const float* gin, float* gout, const float* hin,
                           float* hout, const float* pin, float* pout, const float* phiu_in,
                           float* phiu_out, float* fields, hipStream_t st) {
    const int ntx = (m.nx + TX - 1) / TX, nty = (m.ny + TY - 1) / TY, nch = (m.nz + cz - 1) / cz;
    const long long nblk = (long long)ntx * nty * nch;
    if (nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
    const size_t lds = sizeof(Lds3<TX, TY, PF>);
    static bool attr_set = false;  // dynamic LDS above 64 KiB is requested once per kernel
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&march3d_kernel<TX, TY, C, BC, PF>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((march3d_kernel<TX, TY, C, BC, PF>), dim3((unsigned)nblk), dim3(TX * TY), lds, st, m,
                       gin, gout, hin, hout, pin, pout, phiu_in, phiu_out, fields, ntx, nty, cz);
    return hipGetLastError();
}

template <bool C, int BC>
static hipError_t launch_shape(int s, const Model3& m, const float* gin, float* gout, const float* hin,
                               float* hout, const float* pin, float* pout, const float* phiu_in,
                               float* phiu_out, float* fields, hipStream_t st) {
    const Shape3 sh = kShapes3[s];
#define LBPF3D_CASE(TX, TY)                                                                         \
    if (sh.tx == TX && sh.ty == TY)                                                                 \
        return sh.pf ? launch_t<TX, TY, C, BC, 1>(m, sh.cz, gin, gout, hin, hout, pin, pout, phiu_in, phiu_out, fields, st) \
                     : launch_t<TX, TY, C, BC, 0>(m, sh.cz, gin, gout, hin, hout, pin, pout, phiu_in, phiu_out, fields, st);
    LBPF3D_CASE(32, 8)
    LBPF3D_CASE(64, 4)
    LBPF3D_CASE(64, 8)
    LBPF3D_CASE(32, 16)
#undef LBPF3D_CASE
    return hipErrorInvalidValue;
}

}  // namespace d3q15

// =============================================================================================
// C ABI
// =============================================================================================
using namespace d3q15;

struct lbpf3d {
    lbpf3d_params prm;
    Model3 m;
    float* ws;
    double* red;
    hipStream_t stream;
    int cur;          // which population copy holds the current state (0: A, 1: B)
    int shape;
    int initialized;
    int64_t step;
    std::string err;
};

static thread_local std::string g3_create_error;

static lbpf_status fail3(lbpf3d* c, lbpf_status s, const std::string& msg) {
    if (c) c->err = msg;
    else g3_create_error = msg;
    return s;
}

static lbpf_status hip3(lbpf3d* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return LBPF_OK;
    return fail3(c, LBPF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int pitch3(int nx) { return (nx + 63) / 64 * 64; }

static std::string validate3(const lbpf3d_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return "nx, ny, nz must be >= 3";
    if (p->nx >= (1 << 24) || p->ny >= (1 << 24) || p->nz >= (1 << 24)) return "grid side >= 2^24";
    // row offsets y * pitch use the 24-bit multiplier: the row stride must stay below 2^24
    // floats (interleaved3() falls back to separate planes, whose stride is pitch3(nx))
    if (pitch3(p->nx) >= (1 << 24)) return "nx rounded up to a multiple of 64 must be below 2^24";
    const long long slab = (long long)p->ny * pitch3(p->nx);
    if (slab * p->nz + kPlanePad >= (1LL << 30)) return "nz * ny * pitch(nx) + pad must be < 2^30";
    if (p->variant != 0 && p->variant != 1) return "variant must be 0 (QIM) or 1 (IM)";
    if (p->pscheme < 0 || p->pscheme > 2) return "pscheme must be 0, 1 or 2";
    if (p->fsurf != 0 && p->fsurf != 1) return "fsurf must be 0 or 1";
    if (p->visc != 0 && p->visc != 1) return "visc must be 0 or 1";
    if (p->bc != LBPF3D_BC_PERIODIC && p->bc != LBPF3D_BC_WALLS_Z) return "bc must be 0 or 1";
    if (!(p->tau_h > 0.5)) return "tau_h must be > 1/2";
    if (!(p->nu_A > 0.0) || !(p->nu_B > 0.0)) return "viscosities must be > 0";
    if (!(p->rho_A > 0.0) || !(p->rho_B > 0.0)) return "densities must be > 0";
    if (!(p->W > 0.0)) return "W must be > 0";
    if (!(p->sigma >= 0.0)) return "sigma must be >= 0";
    if (!(p->M_phi >= 0.0)) return "M_phi must be >= 0";
    return "";
}

// Interleaved by row, consecutive planes of a row are pitch3(nx) + 32 floats apart: a row of a
// 256-wide grid is 1 KiB, and planes a power of two apart measured 14.6 GLUPS at 256^3 against
// 17.3 with 32 more floats (17.0 with 64, 128 or 192).
static long long row_plane3(int nx) { return pitch3(nx) + 32; }
static bool interleaved3(const lbpf3d_params* p) {
    const char* e = getenv("LBPF_STATE_LAYOUT");
    if (e && strcmp(e, "planar") == 0) return false;
    const long long stride = kCopyPlanes * row_plane3(p->nx);
    return stride < (1LL << 24) && (long long)p->nz * p->ny * stride < (1LL << 30);
}
static size_t copy_floats3(const lbpf3d_params* p) {
    const size_t rows = (size_t)p->nz * p->ny;
    return interleaved3(p) ? kCopyPlanes * rows * row_plane3(p->nx) + kPlanePad
                           : kCopyPlanes * (rows * pitch3(p->nx) + kPlanePad);
}

static float* copy3(lbpf3d* c, int k) { return c->ws + (size_t)k * c->m.copy; }

// one launch of the march from copy src: a step into the other copy (C), or the field evaluation
// of copy src into the other copy's first seven planes (!C)
template <bool C>
static lbpf_status run3(lbpf3d* c, int src) {
    const Model3& m = c->m;
    const long long P = m.plane;
    const float* in = copy3(c, src);
    float* out = copy3(c, 1 - src);
    float* gout = C ? out + kCopyG * P : nullptr;
    float* hout = C ? out + kCopyH * P : nullptr;
    float* pout = C ? out + kCopyP * P : nullptr;
    float* puout = C ? out + kCopyPhiU * P : nullptr;
    float* fields = C ? nullptr : out;
    hipError_t e = (m.bc == 0)
        ? launch_shape<C, 0>(c->shape, m, in + kCopyG * P, gout, in + kCopyH * P, hout, in + kCopyP * P,
                             pout, in + kCopyPhiU * P, puout, fields, c->stream)
        : launch_shape<C, 1>(c->shape, m, in + kCopyG * P, gout, in + kCopyH * P, hout, in + kCopyP * P,
                             pout, in + kCopyPhiU * P, puout, fields, c->stream);
    return hip3(c, e, "march3d_kernel");
}

extern "C" {

lbpf_status lbpf3d_workspace_size(const lbpf3d_params* params, size_t* bytes) {
    if (!bytes) return fail3(nullptr, LBPF_E_INVALID, "bytes is NULL");
    const std::string v = validate3(params);
    if (!v.empty()) return fail3(nullptr, LBPF_E_INVALID, v);
    const size_t fl = 2 * copy_floats3(params);
    *bytes = (fl * sizeof(float) + 255) / 256 * 256 + kRedDoubles * sizeof(double);
    return LBPF_OK;
}

lbpf_status lbpf3d_create(const lbpf3d_params* params, void* workspace, size_t workspace_bytes,
                          void* hip_stream, lbpf3d** out) {
    if (!out) return fail3(nullptr, LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    const std::string v = validate3(params);
    if (!v.empty()) return fail3(nullptr, LBPF_E_INVALID, v);
    size_t need = 0;
    lbpf3d_workspace_size(params, &need);
    if (!workspace) return fail3(nullptr, LBPF_E_INVALID, "workspace is NULL");
    if (workspace_bytes < need) return fail3(nullptr, LBPF_E_NOMEM, "workspace smaller than lbpf3d_workspace_size");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail3(nullptr, LBPF_E_INVALID, "workspace must be 256-byte aligned");
    lbpf3d* c = new (std::nothrow) lbpf3d();
    if (!c) return fail3(nullptr, LBPF_E_NOMEM, "host allocation failed");
    c->prm = *params;
    c->ws = static_cast<float*>(workspace);
    const size_t fl = 2 * copy_floats3(params);
    c->red = reinterpret_cast<double*>(reinterpret_cast<char*>(workspace) + (fl * sizeof(float) + 255) / 256 * 256);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->shape = kDefaultShape3;
    Model3& m = c->m;
    const lbpf3d_params& p = *params;
    m.nx = p.nx; m.ny = p.ny; m.nz = p.nz;
    const int xp = pitch3(p.nx);
    if (interleaved3(params)) {
        m.plane = row_plane3(p.nx);
        m.pitch = (int)(kCopyPlanes * m.plane);
    } else {
        m.pitch = xp;
        m.plane = (long long)p.nz * p.ny * xp + kPlanePad;
    }
    m.slab = p.ny * m.pitch;
    m.copy = (long long)copy_floats3(params);
    m.variant = p.variant; m.pscheme = p.pscheme; m.fsurf = p.fsurf; m.visc = p.visc;
    m.bc = p.bc; m.clamp = p.clamp_props ? 1 : 0;
    // eqs. (6)-(7): kappa / beta = W^2 / 8, kappa beta = 18 sigma^2
    const double kb = 18.0 * p.sigma * p.sigma, kob = p.W * p.W / 8.0;
    const double kappa = std::sqrt(kb * kob), beta = std::sqrt(kb / kob);
    m.beta4 = (float)(4.0 * beta);
    m.kappa = (float)kappa;
    m.eta = (float)(p.M_phi / ((1.0 / 3.0) * (p.tau_h - 0.5)));  // eq. (17)
    m.gammaM = (float)((p.rho_A - p.rho_B) / p.rho_B * p.M_phi);  // Sec. 3.2.1
    m.rhoA = (float)p.rho_A; m.rhoB = (float)p.rho_B; m.drho = (float)(p.rho_A - p.rho_B);
    m.inv_nuA = (float)(1.0 / p.nu_A); m.inv_nuB = (float)(1.0 / p.nu_B);
    m.muA = (float)(p.rho_A * p.nu_A); m.muB = (float)(p.rho_B * p.nu_B);
    m.inv_tau_h = (float)(1.0 / p.tau_h);
    m.src_coef = (float)(1.0 - 0.5 / p.tau_h);
    m.fx = (float)p.force_x; m.fy = (float)p.force_y; m.fz = (float)p.force_z; m.grav = (float)p.gravity;
    m.d_rhoA = p.rho_A; m.d_rhoB = p.rho_B; m.d_beta = beta; m.d_kappa = kappa;
    *out = c;
    return LBPF_OK;
}

lbpf_status lbpf3d_init(lbpf3d* c, const float* phi, const float* ux, const float* uy, const float* uz,
                        const float* p) {
    if (!c) return LBPF_E_INVALID;
    if (!phi) return fail3(c, LBPF_E_INVALID, "phi is NULL");
    const Model3& m = c->m;
    dim3 grid((m.nx + 255) / 256, m.ny, m.nz);
    if (m.bc == 0)
        hipLaunchKernelGGL(init3d_kernel<0>, grid, dim3(256), 0, c->stream, m, phi, ux, uy, uz, p,
                           copy3(c, 0) + kCopyG * m.plane, copy3(c, 0) + kCopyH * m.plane,
                           copy3(c, 0) + kCopyP * m.plane, copy3(c, 0) + kCopyPhiU * m.plane);
    else
        hipLaunchKernelGGL(init3d_kernel<1>, grid, dim3(256), 0, c->stream, m, phi, ux, uy, uz, p,
                           copy3(c, 0) + kCopyG * m.plane, copy3(c, 0) + kCopyH * m.plane,
                           copy3(c, 0) + kCopyP * m.plane, copy3(c, 0) + kCopyPhiU * m.plane);
    lbpf_status s = hip3(c, hipGetLastError(), "init3d_kernel");
    if (s != LBPF_OK) return s;
    c->cur = 0;
    c->step = 0;
    c->initialized = 1;
    return LBPF_OK;
}

lbpf_status lbpf3d_step(lbpf3d* c, int64_t nsteps) {
    if (!c) return LBPF_E_INVALID;
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "step before init");
    if (nsteps < 0) return fail3(c, LBPF_E_INVALID, "nsteps < 0");
    for (int64_t t = 0; t < nsteps; ++t) {
        lbpf_status s = run3<true>(c, c->cur);
        if (s != LBPF_OK) return s;
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return LBPF_OK;
}

lbpf_status lbpf3d_read(lbpf3d* c, int32_t field, float* dst) {
    if (!c) return LBPF_E_INVALID;
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "read before init");
    if (field < 0 || field >= kNumFields) return fail3(c, LBPF_E_INVALID, "unknown field");
    if (!dst) return fail3(c, LBPF_E_INVALID, "dst is NULL");
    lbpf_status s = run3<false>(c, c->cur);
    if (s != LBPF_OK) return s;
    const Model3& m = c->m;
    hipLaunchKernelGGL(compact3d_kernel, dim3((m.nx + 255) / 256, m.ny, m.nz), dim3(256), 0, c->stream, m,
                       copy3(c, 1 - c->cur) + field * m.plane, dst);
    return hip3(c, hipGetLastError(), "compact3d_kernel");
}

lbpf_status lbpf3d_diagnostics(lbpf3d* c, lbpf_diag* out) {
    if (!c) return LBPF_E_INVALID;
    if (!out) return fail3(c, LBPF_E_INVALID, "out is NULL");
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "diagnostics before init");
    lbpf_status s = run3<false>(c, c->cur);
    if (s != LBPF_OK) return s;
    const Model3& m = c->m;
    const long long n = (long long)m.nx * m.ny * m.nz;
    const int nblk = (int)std::min<long long>(kRedBlocks, (n + 255) / 256);
    const int cur = c->cur;
    hipLaunchKernelGGL(diag3d_partial_kernel, dim3(nblk), dim3(256), 0, c->stream, m,
                       copy3(c, cur) + kCopyG * m.plane, copy3(c, cur) + kCopyH * m.plane,
                       copy3(c, cur) + kCopyP * m.plane, copy3(c, cur) + kCopyPhiU * m.plane,
                       copy3(c, 1 - cur), c->red);
    if ((s = hip3(c, hipGetLastError(), "diag3d_partial_kernel")) != LBPF_OK) return s;
    double* fin = c->red + (size_t)kRedBlocks * kRedSlots;
    hipLaunchKernelGGL(reduce3d_final_kernel, dim3(1), dim3(256), 0, c->stream, c->red, nblk, 1u << 2, fin);
    if ((s = hip3(c, hipGetLastError(), "reduce3d_final_kernel")) != LBPF_OK) return s;
    double h[kRedSlots];
    if ((s = hip3(c, hipMemcpyAsync(h, fin, sizeof(h), hipMemcpyDeviceToHost, c->stream), "copy")) != LBPF_OK)
        return s;
    if ((s = hip3(c, hipStreamSynchronize(c->stream), "sync")) != LBPF_OK) return s;
    out->sum_phi = h[0];
    out->sum_rho = h[1];
    out->max_u = h[2];
    out->nonfinite = (int64_t)h[3];
    out->step = c->step;
    return out->nonfinite ? fail3(c, LBPF_E_UNSTABLE, "non-finite value in the state") : LBPF_OK;
}

lbpf_status lbpf3d_laplace_dp(lbpf3d* c, double xc, double yc, double zc, double R, double* dP) {
    if (!c) return LBPF_E_INVALID;
    if (!dP) return fail3(c, LBPF_E_INVALID, "dP is NULL");
    if (!(R > 0.0)) return fail3(c, LBPF_E_INVALID, "R must be > 0");
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "laplace_dp before init");
    lbpf_status s = run3<false>(c, c->cur);
    if (s != LBPF_OK) return s;
    const Model3& m = c->m;
    const long long n = (long long)m.nx * m.ny * m.nz;
    const int nblk = (int)std::min<long long>(kRedBlocks, (n + 255) / 256);
    const float* h = copy3(c, c->cur) + kCopyH * c->m.plane;
    const double r_in = 0.5 * R, r_out = R + 3.0 * c->prm.W;
    if (m.bc == 0)
        hipLaunchKernelGGL(laplace3d_partial_kernel<0>, dim3(nblk), dim3(256), 0, c->stream, m, h,
                           copy3(c, 1 - c->cur), xc, yc, zc, r_in, r_out, c->red);
    else
        hipLaunchKernelGGL(laplace3d_partial_kernel<1>, dim3(nblk), dim3(256), 0, c->stream, m, h,
                           copy3(c, 1 - c->cur), xc, yc, zc, r_in, r_out, c->red);
    if ((s = hip3(c, hipGetLastError(), "laplace3d_partial_kernel")) != LBPF_OK) return s;
    double* fin = c->red + (size_t)kRedBlocks * kRedSlots;
    hipLaunchKernelGGL(reduce3d_final_kernel, dim3(1), dim3(256), 0, c->stream, c->red, nblk, 0u, fin);
    if ((s = hip3(c, hipGetLastError(), "reduce3d_final_kernel")) != LBPF_OK) return s;
    double r[kRedSlots];
    if ((s = hip3(c, hipMemcpyAsync(r, fin, sizeof(r), hipMemcpyDeviceToHost, c->stream), "copy")) != LBPF_OK)
        return s;
    if ((s = hip3(c, hipStreamSynchronize(c->stream), "sync")) != LBPF_OK) return s;
    if (r[1] < 1.0 || r[3] < 1.0) return fail3(c, LBPF_E_INVALID, "empty inner or outer region");
    *dP = r[0] / r[1] - r[2] / r[3];
    return LBPF_OK;
}

int32_t lbpf3d_shape_count(void) { return kNumShapes3; }

lbpf_status lbpf3d_shape_info(int32_t shape, int32_t* tx, int32_t* ty, int32_t* cz) {
    if (shape < 0 || shape >= kNumShapes3) return fail3(nullptr, LBPF_E_INVALID, "shape out of range");
    if (tx) *tx = kShapes3[shape].tx;
    if (ty) *ty = kShapes3[shape].ty;
    if (cz) *cz = kShapes3[shape].cz;
    return LBPF_OK;
}

lbpf_status lbpf3d_set_shape(lbpf3d* c, int32_t shape) {
    if (!c) return LBPF_E_INVALID;
    if (shape < 0 || shape >= kNumShapes3) return fail3(c, LBPF_E_INVALID, "shape out of range");
    c->shape = shape;
    return LBPF_OK;
}

int32_t lbpf3d_get_shape(const lbpf3d* c) { return c ? c->shape : -1; }

// Time every launch shape for `steps` steps on the current state and keep the fastest. The
// state advances by all the steps taken; every shape gives bit-identical results.
// checkpoint: 64-byte header {magic, version, nx, ny, nz, step, plane stride, copy floats}, then
// the population copy holding the state, as stored
static const int64_t kMagic3 = 0x4433424C;  // "LB3D"
static const int64_t kVersion3 = 1;

lbpf_status lbpf3d_state_size(const lbpf3d* c, size_t* bytes) {
    if (!c || !bytes) return LBPF_E_INVALID;
    *bytes = 64 + (size_t)c->m.copy * sizeof(float);
    return LBPF_OK;
}

lbpf_status lbpf3d_save_state(lbpf3d* c, void* dst) {
    if (!c) return LBPF_E_INVALID;
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "save before init");
    if (!dst) return fail3(c, LBPF_E_INVALID, "dst is NULL");
    const int64_t hdr[8] = {kMagic3, kVersion3, c->m.nx, c->m.ny, c->m.nz, c->step, c->m.plane, c->m.copy};
    lbpf_status s;
    // the header is copied synchronously (it lives on this stack frame)
    if ((s = hip3(c, hipStreamSynchronize(c->stream), "sync")) != LBPF_OK) return s;
    if ((s = hip3(c, hipMemcpy(dst, hdr, sizeof hdr, hipMemcpyHostToDevice), "save header")) != LBPF_OK) return s;
    return hip3(c, hipMemcpyAsync((char*)dst + 64, copy3(c, c->cur), (size_t)c->m.copy * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream), "save state");
}

lbpf_status lbpf3d_load_state(lbpf3d* c, const void* src) {
    if (!c) return LBPF_E_INVALID;
    if (!src) return fail3(c, LBPF_E_INVALID, "src is NULL");
    int64_t hdr[8];
    lbpf_status s;
    if ((s = hip3(c, hipStreamSynchronize(c->stream), "sync")) != LBPF_OK) return s;
    if ((s = hip3(c, hipMemcpy(hdr, src, sizeof hdr, hipMemcpyDeviceToHost), "load header")) != LBPF_OK) return s;
    if (hdr[0] != kMagic3 || hdr[1] != kVersion3 || hdr[2] != c->m.nx || hdr[3] != c->m.ny ||
        hdr[4] != c->m.nz || hdr[6] != c->m.plane || hdr[7] != c->m.copy)
        return fail3(c, LBPF_E_INVALID, "checkpoint does not match this grid and layout");
    c->cur = 0;
    if ((s = hip3(c, hipMemcpyAsync(copy3(c, 0), (const char*)src + 64, (size_t)c->m.copy * sizeof(float),
                                    hipMemcpyDeviceToDevice, c->stream), "load state")) != LBPF_OK)
        return s;
    c->step = hdr[5];
    c->initialized = 1;
    return LBPF_OK;
}

lbpf_status lbpf3d_autotune(lbpf3d* c, int32_t steps, void* scratch_state, int32_t* best_shape) {
    if (!c) return LBPF_E_INVALID;
    if (!c->initialized) return fail3(c, LBPF_E_STATE, "autotune before init");
    if (steps < 1) return fail3(c, LBPF_E_INVALID, "steps < 1");
    hipEvent_t e0, e1;
    lbpf_status s;
    const int64_t step0 = c->step;
    if (scratch_state && (s = lbpf3d_save_state(c, scratch_state)) != LBPF_OK) return s;
    if ((s = hip3(c, hipEventCreate(&e0), "event")) != LBPF_OK) return s;
    if ((s = hip3(c, hipEventCreate(&e1), "event")) != LBPF_OK) { (void)hipEventDestroy(e0); return s; }
    float best = 1e30f;
    int bi = c->shape;
    for (int k = 0; k < kNumShapes3 && s == LBPF_OK; ++k) {
        c->shape = k;
        s = lbpf3d_step(c, 1);  // warm-up of this shape
        if (s != LBPF_OK) break;
        if ((s = hip3(c, hipEventRecord(e0, c->stream), "event")) != LBPF_OK) break;
        if ((s = lbpf3d_step(c, steps)) != LBPF_OK) break;
        if ((s = hip3(c, hipEventRecord(e1, c->stream), "event")) != LBPF_OK) break;
        if ((s = hip3(c, hipEventSynchronize(e1), "event")) != LBPF_OK) break;
        float ms = 0.0f;
        if ((s = hip3(c, hipEventElapsedTime(&ms, e0, e1), "event")) != LBPF_OK) break;
        if (ms < best) { best = ms; bi = k; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->shape = bi;
    if (best_shape) *best_shape = bi;
    if (s != LBPF_OK) return s;
    if (scratch_state) {  // the trial steps are undone: state and step count as on entry
        if ((s = lbpf3d_load_state(c, scratch_state)) != LBPF_OK) return s;
        c->step = step0;
    }
    return LBPF_OK;
}

int64_t lbpf3d_step_count(const lbpf3d* c) { return c ? c->step : -1; }

lbpf_status lbpf3d_destroy(lbpf3d* c) {
    delete c;
    return LBPF_OK;
}

const char* lbpf3d_last_error(const lbpf3d* c) {
    return c ? c->err.c_str() : g3_create_error.c_str();
}

}  // extern "C"
