// Model constants, lattice conventions and device-workspace layout of the lbpf library.
// Host and device code both include this header; it holds no arithmetic of the method beyond
// the D2Q9 lattice definition (Sec. 2.2 of arXiv:1902.08933, listed after eq. 25).
#pragma once

#include <cstddef>
#include <cstdint>

namespace lbpf {

// D2Q9 velocity order of the paper: 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+1,+1), 6 (-1,+1),
// 7 (-1,-1), 8 (+1,-1); weights 4/9, 1/9 (axes), 1/36 (diagonals); c_s^2 = 1/3.
constexpr int kQ = 9;

// Per-cell stored planes of one population copy. The hydrodynamic distribution keeps
// directions 1..8 only: its rest population never enters any output of the two-phase model
// (u uses c_0 = 0, eq. (28) sums i != 0, rho comes from phi). The phase-field distribution
// keeps all nine directions; its rest population carries the order parameter and is stored
// as an unevaluated FP32 sum hi + lo.
constexpr int kFPlanes = 8;   // f_1..f_8   -> plane i-1
constexpr int kHPlanes = 10;  // h_0 hi, h_1..h_8, h_0 lo -> planes 0, 1..8, 9
constexpr int kH0Lo = 9;

// One population copy (the state at one time level) holds 21 planes:
//   0..7    f_1..f_8
//   8..17   h_0 hi, h_1..h_8, h_0 lo
//   18      p
//   19, 20  (phi u)_x, (phi u)_y
// The workspace holds two copies (a step reads one and writes the other), then an FP64 scratch
// of ny * xpitch doubles (order parameter in double for the Laplace diagnostic), then the
// reduction area (kRedDoubles doubles). Between steps the copy that does not hold the state is
// free: field evaluation (phi, rho, ux, uy, p, mu for reads, diagnostics and the hand-over to the
// surrogate) writes its six planes there.
//
// Element (q, y, x) of a copy sits at q * plane + y * pitch + x. The planes are either
// interleaved by grid row (pitch = 21 xpitch, plane = xpitch: the 21 values of a row of nodes are
// neighbours in memory, so a workgroup keeps few DRAM pages open) or separate (pitch = xpitch,
// plane = ny * xpitch + pad) for grids too large for 32-bit per-lane offsets when interleaved.
constexpr int kCopyF = 0, kCopyH = 8, kCopyP = 18, kCopyPhiU = 19, kCopyPlanes = 21;
constexpr int kFieldPlanes = 6;
constexpr int kRedBlocks = 4096;                 // max partial-sum blocks of a reduction
constexpr int kRedSlots = 8;                     // doubles per partial
constexpr size_t kRedDoubles = (size_t)kRedBlocks * kRedSlots + 64;

inline int pitch_of(int nx) { return (nx + 63) / 64 * 64; }
constexpr long kDefaultPlanePad = 4160;  // floats; measured +5..10 % at 4096^2, neutral at 1024^2

// Physical and derived model constants in the precision the kernels compute in (FP32).
struct Model {
    int nx, ny;
    int pitch;             // floats between rows of a copy (row stride)
    int xpitch;            // floats per row of one plane: nx rounded up to 64
    long long plane;       // floats between planes of a copy
    long long copy;        // floats per population copy (21 planes and a pad)
    int variant;           // 0 quasi-incompressible, 1 incompressible
    int pscheme;           // 0 eq.(28) with G0 of eq.(34), 1 simplified G0, 2 eq.(29)
    int fsurf;             // 0 mu grad phi, 1 -phi grad mu
    int visc;              // 0 inverse-linear, 1 step
    int bc;                // 0 periodic, 1 walls in y
    int clamp;             // clamp phi to [0,1] in rho(phi), nu(phi)
    float beta4;           // 4 beta, beta = 12 sigma / W   (eqs. 6-7)
    float kappa;           // kappa = 3 sigma W / 2          (eqs. 6-7)
    float eta;             // M_phi / (c_s^2 (tau_h - 1/2))  (eq. 17)
    float gammaM;          // gamma M_phi, gamma = (rho_A - rho_B)/rho_B (Sec. 3.2.1)
    float rhoA, rhoB, drho;
    float inv_nuA, inv_nuB; // inverse-linear viscosity
    float muA, muB;         // dynamic viscosities for the step form
    float inv_tau_h;
    float src_coef;         // 1 - 1/(2 tau_h) of eq. (14)
    float fx, fy, grav;
    // FP64 copies for the diagnostics
    double d_beta, d_kappa, d_rhoA, d_rhoB;
};

// One simulation of a batch, as the batched kernel sees it (device memory).
struct BatchInst {
    Model m;
    long long ws_off;  // the instance's workspace (population copies as above), in floats from
                       // the start of the batch's workspace
    int nsx, nsy;     // strips and chunks of the batch's strip shape
};
// Counter slots of the batched kernel (launches use them in cyclic order; see batch_kernel).
constexpr int kBatchSlots = 8;
// One unit of work of the batched kernel: chunk `chunk` (row-major over nsx x nsy) of `inst`.
struct BatchItem {
    int inst, chunk;
};

// Deterministic reduction results (FP64).
struct DiagOut {
    double sum_phi, sum_rho, max_u, nonfinite;
};

}  // namespace lbpf
