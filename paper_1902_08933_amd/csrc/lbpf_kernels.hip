// HIP kernels of the lbpf library for gfx950 (MI355X).
//
// One time step of the phase-field lattice Boltzmann model of arXiv:1902.08933, Sec. 3, is one
// launch of fused_kernel<..., true>. The stored state is the pair of distributions after
// streaming (the paper's g_i(x,t), h_i(x,t)); the kernel computes all macroscopic quantities of
// time t, collides (eq. 24, eq. 10) and pushes the post-collision populations to x + c_i in the
// other copy (periodic wrap, or halfway bounce-back at y walls).
//
// Per launch, a workgroup owns a TX x TY tile and stages in LDS:
//   phi  on the tile plus a ring of 2 (needed by lap(phi) of mu on the ring of 1 and by
//        grad(phi) on the tile), as an FP32 hi/lo pair: phi = sum_i h_i (eq. 18) where h_0 is
//        stored as hi + lo, so phi keeps ~48 significant bits through the stencils;
//   mu   on the tile plus a ring of 1 (eq. 8 with the Laplacian of eq. 30b);
//   p    of the previous step on the tile plus a ring of 1 (its gradient enters F~).
// Everything else is FP32 arithmetic in registers. Each cell moves 168 bytes of HBM traffic:
// f_1..8, h_0 hi, h_1..8, h_0 lo, p, (phi u)_x,y read once and written once.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbpf_model.hpp"

namespace lbpf {

// D2Q9 (Sec. 2.2, listed after eq. 25)
__device__ constexpr int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float kW0 = 4.0f / 9.0f, kWA = 1.0f / 9.0f, kWD = 1.0f / 36.0f;
__device__ __forceinline__ constexpr float wgt(int q) { return q == 0 ? kW0 : (q < 5 ? kWA : kWD); }

// Error-free transformation of a sum (Knuth): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ int wrap(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Row read for a stencil ghost: periodic wrap, or the mirror image about a wall half a cell
// outside the first/last fluid row (clamped for rows that no active cell reads).
__device__ __forceinline__ int src_row(int y, int ny, int bc) {
    if (bc == 0) return wrap(y, ny);
    if (y < 0) y = -1 - y;
    else if (y >= ny) y = 2 * ny - 1 - y;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
}

// XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs, so block b runs on
// XCD b % 8. Give each XCD a contiguous band of tiles so that the halos shared by neighbouring
// tiles are re-read from the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
    const int per = nblk / 8, rem = nblk % 8, xcd = b % 8, loc = b / 8;
    return xcd * per + (xcd < rem ? xcd : rem) + loc;
}

// ---------------------------------------------------------------------------------------------
// Fused step (COLLIDE = true) and field evaluation (COLLIDE = false)
// ---------------------------------------------------------------------------------------------
template <int TX, int TY, int NT, bool COLLIDE>
__global__ __launch_bounds__(NT) void fused_kernel(Model m, const float* __restrict__ fin,
                                                   float* __restrict__ fout,
                                                   const float* __restrict__ hin,
                                                   float* __restrict__ hout,
                                                   const float* __restrict__ pin,
                                                   float* __restrict__ pout,
                                                   float* __restrict__ phiu,
                                                   float* __restrict__ fields, int ntx, int nty) {
    constexpr int PX = TX + 4, PY = TY + 4;  // phi tile, ring of 2
    constexpr int MX = TX + 2, MY = TY + 2;  // mu and p tiles, ring of 1
    constexpr int RPP = NT / TX;             // tile rows per pass of the workgroup
    constexpr int OWN = TY / RPP;            // cells per thread
    static_assert(NT % TX == 0 && TY % RPP == 0, "tile/thread mapping");
    __shared__ float s_phh[PY * PX];
    __shared__ float s_phl[PY * PX];
    __shared__ float s_mu[MY * MX];
    __shared__ float s_p[MY * MX];

    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int tid = threadIdx.x;
    const long long P = m.plane;
    const int pitch = m.pitch, nx = m.nx, ny = m.ny;

    // ---- phase 1: phi = sum_i h_i (eq. 18) on the tile + 2 ring, hi/lo pair ----------------
    for (int i = tid; i < PX * PY; i += NT) {
        const int lx = i % PX, ly = i / PX;
        const int sx = wrap(x0 + lx - 2, nx), sy = src_row(y0 + ly - 2, ny, m.bc);
        const float* hp = hin + (long long)sy * pitch + sx;
        float s = 0.0f;
#pragma unroll
        for (int q = 1; q <= 8; ++q) s += hp[q * P];
        float ph, e;
        two_sum(hp[0], s, ph, e);
        s_phh[i] = ph;
        s_phl[i] = hp[kH0Lo * P] + e;
    }
    __syncthreads();

    // ---- phase 2: mu (eq. 8) and the previous pressure on the tile + 1 ring ----------------
    for (int i = tid; i < MX * MY; i += NT) {
        const int lx = i % MX, ly = i / MX;
        const int gx = x0 + lx - 1, gy = y0 + ly - 1;
        int cy = gy;  // a ghost row beyond a wall takes the value of its mirror row
        if (m.bc == 1) {
            if (gy < 0) cy = -1 - gy;
            else if (gy >= ny) cy = 2 * ny - 1 - gy;
        }
        const int py = cy - y0 + 2, px = lx + 1;
        float mu = 0.0f;
        if (py >= 1 && py <= PY - 2) {
            const int c = py * PX + px;
            const float ch = s_phh[c], cl = s_phl[c];
            // differences of neighbours in hi/lo form keep the full precision of phi
            auto d = [&](int o) { return (s_phh[c + o] - ch) + (s_phl[c + o] - cl); };
            const float axes = (d(1) + d(-1)) + (d(PX) + d(-PX));
            const float diag = (d(PX + 1) + d(PX - 1)) + (d(-PX + 1) + d(-PX - 1));
            const float lap = (2.0f / 3.0f) * axes + (1.0f / 6.0f) * diag;  // eq. (30b)
            const float a = ch + cl, b = (ch - 1.0f) + cl, cc = (ch - 0.5f) + cl;
            mu = m.beta4 * a * b * cc - m.kappa * lap;
        }
        s_mu[i] = mu;
        s_p[i] = pin[(long long)src_row(gy, ny, m.bc) * pitch + wrap(gx, nx)];
    }
    __syncthreads();

    // ---- phase 3: per owned cell ------------------------------------------------------------
    const int tx = tid % TX, ty0 = tid / TX;
    for (int k = 0; k < OWN; ++k) {
        const int ly = ty0 + k * RPP;
        const int x = x0 + tx, y = y0 + ly;
        if (x >= nx || y >= ny) continue;
        const long long cell = (long long)y * pitch + x;

        // isotropic stencils, eq. (30a) and eq. (30b)
        const int pc = (ly + 2) * PX + (tx + 2);
        const float ch = s_phh[pc], cl = s_phl[pc];
        auto dphi = [&](int oa, int ob) {
            return (s_phh[pc + oa] - s_phh[pc + ob]) + (s_phl[pc + oa] - s_phl[pc + ob]);
        };
        // grad z = (z_E - z_W)/3 + (z_NE - z_NW + z_SE - z_SW)/12, y likewise
        const float gphix = (1.0f / 3.0f) * dphi(1, -1)
                          + (1.0f / 12.0f) * (dphi(PX + 1, PX - 1) + dphi(-PX + 1, -PX - 1));
        const float gphiy = (1.0f / 3.0f) * dphi(PX, -PX)
                          + (1.0f / 12.0f) * (dphi(PX + 1, -PX + 1) + dphi(PX - 1, -PX - 1));
        const int mc = (ly + 1) * MX + (tx + 1);
        const float mu = s_mu[mc];
        auto gradc = [&](const float* s, float& gx, float& gy) {
            gx = (1.0f / 3.0f) * (s[mc + 1] - s[mc - 1])
               + (1.0f / 12.0f) * ((s[mc + MX + 1] - s[mc + MX - 1]) + (s[mc - MX + 1] - s[mc - MX - 1]));
            gy = (1.0f / 3.0f) * (s[mc + MX] - s[mc - MX])
               + (1.0f / 12.0f) * ((s[mc + MX + 1] - s[mc - MX + 1]) + (s[mc + MX - 1] - s[mc - MX - 1]));
        };
        float gmux, gmuy, gpx, gpy;
        gradc(s_mu, gmux, gmuy);
        gradc(s_p, gpx, gpy);
        const float lapmu = (2.0f / 3.0f) * (((s_mu[mc + 1] - mu) + (s_mu[mc - 1] - mu))
                                           + ((s_mu[mc + MX] - mu) + (s_mu[mc - MX] - mu)))
                          + (1.0f / 6.0f) * (((s_mu[mc + MX + 1] - mu) + (s_mu[mc + MX - 1] - mu))
                                           + ((s_mu[mc - MX + 1] - mu) + (s_mu[mc - MX - 1] - mu)));

        // populations of this cell
        float f[9], h[9];
#pragma unroll
        for (int q = 1; q <= 8; ++q) f[q] = fin[(q - 1) * P + cell];
        const float h0hi = hin[cell], h0lo = hin[kH0Lo * P + cell];
        float hs = 0.0f;
#pragma unroll
        for (int q = 1; q <= 8; ++q) {
            h[q] = hin[q * P + cell];
            hs += h[q];
        }
        const float pux_prev = phiu[cell], puy_prev = phiu[P + cell];

        // closure: eq. (3aa), viscosity, forces
        const float phi = ch + cl;
        const float phic = m.clamp ? fminf(fmaxf(phi, 0.0f), 1.0f) : phi;
        const float rho = m.rhoB + m.drho * phic;
        float Fx, Fy;
        if (m.fsurf == 0) { Fx = mu * gphix; Fy = mu * gphiy; }
        else { Fx = -phi * gmux; Fy = -phi * gmuy; }
        Fx += m.fx;
        Fy += m.fy - (rho - m.rhoA) * m.grav;
        // eq. (27a): u = (sum_i c_i g_i + F/2) / rho
        const float mx = ((f[1] - f[3]) + (f[5] - f[7])) + (f[8] - f[6]);
        const float my = ((f[2] - f[4]) + (f[5] - f[7])) + (f[6] - f[8]);
        const float ux = (mx + 0.5f * Fx) / rho, uy = (my + 0.5f * Fy) / rho;
        // mass source: S1 = -gamma M lap(mu) (quasi-incompressible) or 0; S = u.grad(rho) + rho S1
        const float S1 = (m.variant == 0) ? -m.gammaM * lapmu : 0.0f;
        const float grx = m.drho * gphix, gry = m.drho * gphiy;
        const float rS1 = rho * S1;
        const float S = (ux * grx + uy * gry) + rS1;
        // F~ = F - grad(p - rho c_s^2) with the previous step's pressure
        const float Ftx = Fx - gpx + (1.0f / 3.0f) * grx, Fty = Fy - gpy + (1.0f / 3.0f) * gry;
        const float uFt = ux * Ftx + uy * Fty;
        // tau_g from nu(phi): nu = c_s^2 (tau_g - 1/2)
        float nu;
        if (m.visc == 0) nu = 1.0f / (phic * (m.inv_nuA - m.inv_nuB) + m.inv_nuB);
        else nu = ((phi >= 0.5f) ? m.muA : m.muB) / rho;
        const float tau_g = 3.0f * nu + 0.5f;
        // eq. (28): p = 3/5 [ sum_{i!=0} g_i + S/2 + rho s_0(u) + (tau_g - 1/2) G_0 ]
        const float u2 = ux * ux + uy * uy;
        const float sumf = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
        float bracket = sumf + 0.5f * S - (2.0f / 3.0f) * rho * u2;
        if (m.pscheme == 0) {
            // eq. (34) at i = 0: G_0 = w_0 (S - u.F~/c_s^2 - rho S1)
            bracket += (tau_g - 0.5f) * (kW0 * (S - 3.0f * uFt - rS1));
        } else if (m.pscheme == 1) {
            const float uFp = ux * (Fx - gpx) + uy * (Fy - gpy);
            bracket += (tau_g - 0.5f) * (kW0 * (0.5f * rS1 - 3.0f * uFp));
        }
        const float p = 0.6f * bracket;
        const float phiux = phi * ux, phiuy = phi * uy;

        if constexpr (!COLLIDE) {
            float* o = fields + cell;
            o[0] = phi;
            o[P] = rho;
            o[2 * P] = ux;
            o[3 * P] = uy;
            o[4 * P] = p;
            o[5 * P] = mu;
            continue;
        } else {
            const float omega = 1.0f / tau_g;
            const float fgain = 1.0f - 0.5f * omega;
            const float emu = m.eta * mu;
            const float dpx = phiux - pux_prev, dpy = phiuy - puy_prev;
            const float rcoef = 3.0f * m.src_coef;
            const float ith = m.inv_tau_h;
            const int xp = (x + 1 == nx) ? 0 : x + 1, xm = (x == 0) ? nx - 1 : x - 1;
            const bool walls = (m.bc == 1);
            const int yp = (y + 1 == ny) ? 0 : y + 1, ym = (y == 0) ? ny - 1 : y - 1;
            const bool wall_top = walls && (y == ny - 1), wall_bot = walls && (y == 0);
#pragma unroll
            for (int q = 1; q <= 8; ++q) {
                const float w = wgt(q);
                const int cx = kCX[q], cy = kCY[q];
                const float cu = cx * ux + cy * uy;
                const float cF = cx * Fx + cy * Fy;
                const float cFt = cx * Ftx + cy * Fty;
                const float c2 = (float)(cx * cx + cy * cy);
                // eq. (34) expanded for d = 2:
                // G_i = w_i [S + c.F/c_s^2 + ((c.u)(c.F~) - c_s^2 u.F~)/c_s^4 + rho S1 (|c|^2 - 2 c_s^2)/(2 c_s^2)]
                const float G = w * (S + 3.0f * cF + 9.0f * cu * cFt - 3.0f * uFt + rS1 * (1.5f * c2 - 1.0f));
                // eq. (33), i != 0: g_i^eq = w_i p / c_s^2 + rho s_i(u)
                const float geq = w * (3.0f * p + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2));
                // eq. (24)
                const float fst = f[q] - (f[q] - geq) * omega + fgain * G;
                // eq. (11), i != 0, and eq. (14)
                const float heq = w * (emu + 3.0f * (cx * phiux + cy * phiuy));
                const float R = rcoef * w * (cx * dpx + cy * dpy);
                // eq. (10)
                const float hst = h[q] - (h[q] - heq) * ith + R;
                // streaming to x + c_i, or back into this cell across a wall
                int dx = cx > 0 ? xp : (cx < 0 ? xm : x);
                int dy = cy > 0 ? yp : (cy < 0 ? ym : y);
                int dq = q;
                if ((cy > 0 && wall_top) || (cy < 0 && wall_bot)) {
                    dx = x;
                    dy = y;
                    dq = kOpp[q];
                }
                const long long dst = (long long)dy * pitch + dx;
                fout[(dq - 1) * P + dst] = fst;
                hout[dq * P + dst] = hst;
            }
            // rest population of h: h_0* = h_0 - (h_0 - h_0^eq)/tau_h with h_0 - h_0^eq
            // = -sum_{i!=0} h_i - (w_0 - 1) eta mu; added to the hi/lo pair without rounding h_0
            const float dh0 = (hs + (kW0 - 1.0f) * emu) * ith;
            float nh, e;
            two_sum(h0hi, dh0, nh, e);
            const float nl = h0lo + e;
            float hi2, lo2;
            two_sum(nh, nl, hi2, lo2);
            hout[cell] = hi2;
            hout[kH0Lo * P + cell] = lo2;
            pout[cell] = p;
            phiu[cell] = phiux;
            phiu[P + cell] = phiuy;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Initial state: equilibria of eq. (11) and eq. (33) at (phi0, mu0, u0, p0)
// ---------------------------------------------------------------------------------------------
__global__ void init_kernel(Model m, const float* __restrict__ phi0, const float* __restrict__ ux0,
                            const float* __restrict__ uy0, const float* __restrict__ p0,
                            float* __restrict__ f, float* __restrict__ h, float* __restrict__ pp,
                            float* __restrict__ phiu) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= m.nx || y >= m.ny) return;
    const int nx = m.nx, ny = m.ny;
    auto at = [&](int dx, int dy) {
        return phi0[(long long)src_row(y + dy, ny, m.bc) * nx + wrap(x + dx, nx)];
    };
    const float c = at(0, 0);
    const float axes = ((at(1, 0) - c) + (at(-1, 0) - c)) + ((at(0, 1) - c) + (at(0, -1) - c));
    const float diag = ((at(1, 1) - c) + (at(-1, 1) - c)) + ((at(1, -1) - c) + (at(-1, -1) - c));
    const float lap = (2.0f / 3.0f) * axes + (1.0f / 6.0f) * diag;
    const float mu = m.beta4 * c * (c - 1.0f) * (c - 0.5f) - m.kappa * lap;
    const long long in = (long long)y * nx + x;
    const float ux = ux0 ? ux0[in] : 0.0f, uy = uy0 ? uy0[in] : 0.0f, p = p0 ? p0[in] : 0.0f;
    const float phic = m.clamp ? fminf(fmaxf(c, 0.0f), 1.0f) : c;
    const float rho = m.rhoB + m.drho * phic;
    const long long cell = (long long)y * m.pitch + x, P = m.plane;
    const float emu = m.eta * mu, u2 = ux * ux + uy * uy;
    const float phiux = c * ux, phiuy = c * uy;
    float hi, lo;
    two_sum(c, (kW0 - 1.0f) * emu, hi, lo);
    h[cell] = hi;
    h[kH0Lo * P + cell] = lo;
#pragma unroll
    for (int q = 1; q <= 8; ++q) {
        const float w = wgt(q);
        const float cu = kCX[q] * ux + kCY[q] * uy;
        f[(q - 1) * P + cell] = w * (3.0f * p + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2));
        h[q * P + cell] = w * (emu + 3.0f * (kCX[q] * phiux + kCY[q] * phiuy));
    }
    pp[cell] = p;
    phiu[cell] = phiux;
    phiu[P + cell] = phiuy;
}

// ---------------------------------------------------------------------------------------------
// FP64 reductions: deterministic two-pass (per-block partials, then one block in fixed order)
// ---------------------------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_reduce(double v, double* sh, bool is_max) {
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
        for (int i = 1; i < NT / 64; ++i) r = is_max ? fmax(r, sh[i]) : r + sh[i];
    }
    return r;
}

// Partials over the stored state of the current copy: sum phi, sum rho, max |u| (from the
// field scratch written by the field kernel), count of non-finite stored values.
__global__ __launch_bounds__(256) void diag_partial_kernel(Model m, const float* __restrict__ f,
                                                           const float* __restrict__ h,
                                                           const float* __restrict__ pp,
                                                           const float* __restrict__ phiu,
                                                           const float* __restrict__ fields,
                                                           double* __restrict__ part) {
    __shared__ double sh[4];
    const long long n = (long long)m.nx * m.ny, P = m.plane;
    double sphi = 0.0, srho = 0.0, umax = 0.0, bad = 0.0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % m.nx), y = (int)(k / m.nx);
        const long long cell = (long long)y * m.pitch + x;
        double phi = (double)h[cell] + (double)h[kH0Lo * P + cell];
        for (int q = 1; q <= 8; ++q) phi += (double)h[q * P + cell];
        double phc = phi;
        if (m.clamp) phc = phc < 0.0 ? 0.0 : (phc > 1.0 ? 1.0 : phc);
        sphi += phi;
        srho += m.d_rhoB + (m.d_rhoA - m.d_rhoB) * phc;
        const double ux = fields[2 * P + cell], uy = fields[3 * P + cell];
        const double um = sqrt(ux * ux + uy * uy);
        umax = (um > umax || um != um) ? um : umax;
        int nb = 0;
        for (int q = 0; q < kFPlanes; ++q) nb += !isfinite(f[q * P + cell]);
        for (int q = 0; q < kHPlanes; ++q) nb += !isfinite(h[q * P + cell]);
        nb += !isfinite(pp[cell]) + !isfinite(phiu[cell]) + !isfinite(phiu[P + cell]);
        bad += nb;
    }
    const double a = block_reduce<256>(sphi, sh, false);
    const double b = block_reduce<256>(srho, sh, false);
    const double c = block_reduce<256>(umax, sh, true);
    const double d = block_reduce<256>(bad, sh, false);
    if (threadIdx.x == 0) {
        double* o = part + (size_t)blockIdx.x * kRedSlots;
        o[0] = a; o[1] = b; o[2] = c; o[3] = d;
    }
}

// Second pass: slot s of every partial reduced by one workgroup in a fixed order.
// maxmask bit s selects max instead of sum for slot s.
__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ part, int nblk,
                                                           int nslots, unsigned maxmask,
                                                           double* __restrict__ out) {
    __shared__ double sh[4];
    for (int s = 0; s < nslots; ++s) {
        const bool is_max = (maxmask >> s) & 1u;
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) {
            const double w = part[(size_t)b * kRedSlots + s];
            v = is_max ? ((w > v || w != w) ? w : v) : v + w;
        }
        const double r = block_reduce<256>(v, sh, is_max);
        if (threadIdx.x == 0) out[s] = r;
    }
}

// phi in FP64 for every node: h_0 hi + h_0 lo + sum_{i!=0} h_i (eq. 18)
__global__ void phi64_kernel(Model m, const float* __restrict__ h, double* __restrict__ phi64) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= m.nx || y >= m.ny) return;
    const long long cell = (long long)y * m.pitch + x, P = m.plane;
    double phi = (double)h[cell] + (double)h[kH0Lo * P + cell];
    for (int q = 1; q <= 8; ++q) phi += (double)h[q * P + cell];
    phi64[cell] = phi;
}

// Laplace pressure of Sec. 4.2 in FP64, P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p
// with p0 = phi psi' - psi, psi = beta phi^2 (phi - 1)^2; partial sums over the inner disc
// r <= r_in and the outer region r >= r_out (periodic distance in periodic directions).
__global__ __launch_bounds__(256) void laplace_partial_kernel(Model m, const double* __restrict__ phi64,
                                                              const float* __restrict__ fields,
                                                              double xc, double yc, double r_in,
                                                              double r_out, double* __restrict__ part) {
    __shared__ double sh[4];
    const long long n = (long long)m.nx * m.ny, P = m.plane;
    double s_in = 0.0, c_in = 0.0, s_out = 0.0, c_out = 0.0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int x = (int)(k % m.nx), y = (int)(k / m.nx);
        auto at = [&](int dx, int dy) {
            return phi64[(long long)src_row(y + dy, m.ny, m.bc) * m.pitch + wrap(x + dx, m.nx)];
        };
        const double c = at(0, 0);
        const double gx = (at(1, 0) - at(-1, 0)) / 3.0 + ((at(1, 1) - at(-1, 1)) + (at(1, -1) - at(-1, -1))) / 12.0;
        const double gy = (at(0, 1) - at(0, -1)) / 3.0 + ((at(1, 1) - at(1, -1)) + (at(-1, 1) - at(-1, -1))) / 12.0;
        const double lap = (2.0 / 3.0) * (((at(1, 0) - c) + (at(-1, 0) - c)) + ((at(0, 1) - c) + (at(0, -1) - c)))
                         + (1.0 / 6.0) * (((at(1, 1) - c) + (at(-1, 1) - c)) + ((at(1, -1) - c) + (at(-1, -1) - c)));
        const double psi = m.d_beta * c * c * (c - 1.0) * (c - 1.0);
        const double dpsi = 4.0 * m.d_beta * c * (c - 1.0) * (c - 0.5);
        const double p0 = c * dpsi - psi;
        const double p = (double)fields[4 * P + (long long)y * m.pitch + x];
        const double Pt = p0 - m.d_kappa * c * lap + 0.5 * m.d_kappa * (gx * gx + gy * gy) + p;
        double dx = fabs(x - xc), dy = fabs(y - yc);
        dx = fmin(dx, m.nx - dx);
        if (m.bc == 0) dy = fmin(dy, m.ny - dy);
        const double r = sqrt(dx * dx + dy * dy);
        if (r <= r_in) { s_in += Pt; c_in += 1.0; }
        if (r >= r_out) { s_out += Pt; c_out += 1.0; }
    }
    const double a = block_reduce<256>(s_in, sh, false);
    const double b = block_reduce<256>(c_in, sh, false);
    const double c = block_reduce<256>(s_out, sh, false);
    const double d = block_reduce<256>(c_out, sh, false);
    if (threadIdx.x == 0) {
        double* o = part + (size_t)blockIdx.x * kRedSlots;
        o[0] = a; o[1] = b; o[2] = c; o[3] = d;
    }
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
struct TileShape { int tx, ty, nt; };
static const TileShape kTiles[] = {{64, 16, 256}, {64, 8, 256}, {64, 32, 256}, {128, 8, 256},
                                   {128, 16, 256}, {32, 16, 128}, {64, 16, 512}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

int tile_count() { return kNumTiles; }
void tile_shape(int i, int* tx, int* ty, int* nt) {
    *tx = kTiles[i].tx; *ty = kTiles[i].ty; *nt = kTiles[i].nt;
}

template <int TX, int TY, int NT, bool C>
static hipError_t launch_fused_t(const Model& m, const float* fin, float* fout, const float* hin,
                                 float* hout, const float* pin, float* pout, float* phiu,
                                 float* fields, hipStream_t st) {
    const int ntx = (m.nx + TX - 1) / TX, nty = (m.ny + TY - 1) / TY;
    hipLaunchKernelGGL((fused_kernel<TX, TY, NT, C>), dim3(ntx * nty), dim3(NT), 0, st, m, fin,
                       fout, hin, hout, pin, pout, phiu, fields, ntx, nty);
    return hipGetLastError();
}

template <bool C>
static hipError_t launch_fused(int tile, const Model& m, const float* fin, float* fout,
                               const float* hin, float* hout, const float* pin, float* pout,
                               float* phiu, float* fields, hipStream_t st) {
    switch (tile) {
        case 0: return launch_fused_t<64, 16, 256, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 1: return launch_fused_t<64, 8, 256, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 2: return launch_fused_t<64, 32, 256, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 3: return launch_fused_t<128, 8, 256, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 4: return launch_fused_t<128, 16, 256, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 5: return launch_fused_t<32, 16, 128, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        case 6: return launch_fused_t<64, 16, 512, C>(m, fin, fout, hin, hout, pin, pout, phiu, fields, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(int tile, const Model& m, const float* fin, float* fout, const float* hin,
                       float* hout, const float* pin, float* pout, float* phiu, hipStream_t st) {
    return launch_fused<true>(tile, m, fin, fout, hin, hout, pin, pout, phiu, nullptr, st);
}

hipError_t launch_fields(const Model& m, const float* fin, const float* hin, const float* pin,
                         float* phiu, float* fields, hipStream_t st) {
    return launch_fused<false>(0, m, fin, nullptr, hin, nullptr, pin, nullptr, phiu, fields, st);
}

hipError_t launch_init(const Model& m, const float* phi0, const float* ux0, const float* uy0,
                       const float* p0, float* f, float* h, float* pp, float* phiu, hipStream_t st) {
    dim3 grid((m.nx + 255) / 256, m.ny);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, st, m, phi0, ux0, uy0, p0, f, h, pp, phiu);
    return hipGetLastError();
}

static int red_blocks(const Model& m) {
    long long n = (long long)m.nx * m.ny;
    long long b = (n + 1023) / 1024;
    if (b > kRedBlocks) b = kRedBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_diag(const Model& m, const float* f, const float* h, const float* pp,
                       const float* phiu, const float* fields, double* red, hipStream_t st) {
    const int nb = red_blocks(m);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(nb), dim3(256), 0, st, m, f, h, pp, phiu, fields, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* out = red + (size_t)kRedBlocks * kRedSlots;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, st, red, nb, 4, 0x4u, out);
    return hipGetLastError();
}

hipError_t launch_laplace(const Model& m, const float* h, const float* fields, double* phi64,
                          double xc, double yc, double r_in, double r_out, double* red,
                          hipStream_t st) {
    dim3 grid((m.nx + 255) / 256, m.ny);
    hipLaunchKernelGGL(phi64_kernel, grid, dim3(256), 0, st, m, h, phi64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = red_blocks(m);
    hipLaunchKernelGGL(laplace_partial_kernel, dim3(nb), dim3(256), 0, st, m, phi64, fields, xc,
                       yc, r_in, r_out, red);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* out = red + (size_t)kRedBlocks * kRedSlots;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, st, red, nb, 4, 0x0u, out);
    return hipGetLastError();
}

}  // namespace lbpf
