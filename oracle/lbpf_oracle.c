/*
 * FP64 CPU oracle for the phase-field lattice Boltzmann model with a mass source of
 * Yuan, Chai, Wang & Shi, "A generalized lattice Boltzmann model for fluid flow system and its
 * application in two-phase flows" (arXiv:1902.08933).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library. It shares no source, header, table or helper with the HIP
 * library: it is written from the paper alone, in plain loops, in double precision, in the
 * order in which the paper states the method. It is deliberately slow and unblocked.
 *
 * Paper map (section / equation labels as printed in the paper):
 *   lattice                 Sec. 2.2, D2Q9 weights and velocities (after eq. 25)
 *   hydrodynamic LB         eq. (24) evolution, eq. (33) equilibrium, eq. (34) force term,
 *                           eq. (27a) velocity, eq. (28) / (29) pressure
 *   phase-field LB          eq. (10) evolution, eq. (11) equilibrium, eq. (14) source,
 *                           first-order time difference below eq. (14), eq. (18) order parameter,
 *                           eq. (17) mobility
 *   closure                 eq. (3aa) density, eq. (8) chemical potential, eqs. (6)-(7) beta and
 *                           kappa, Sec. 3.1 surface tension F_s and S = u.grad(rho) + rho S1,
 *                           Sec. 3.2.1 gamma of the quasi-incompressible source, inverse-linear
 *                           viscosity after eq. (17), step viscosity of Sec. 4.3
 *   stencils                eqs. (30a), (30b)
 *   Laplace diagnostic      Sec. 4.2, P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p
 *
 * Readings where the paper is silent or inconsistent (each is a switch or a documented choice):
 *   G0         eq. (34) evaluated at i = 0 is used by default (pscheme 0); pscheme 1 uses the
 *              simplified G0 printed after eq. (34), which loses the trace factor d;
 *              pscheme 2 is eq. (29) (no G0 term).
 *   grad p     F~ and the paper's simplified G0 need grad p while p needs G0: the gradient of the
 *              previous step's pressure is used; before the first step it is the initial p.
 *   R_i        the relaxation time in eq. (14) is tau_h; (phi u) at the step before the first is
 *              phi0 u0 of the initial fields.
 *   rho_0      the constant in eq. (33) is 1; it only enters g_0, which no output reads.
 *   init       g_i = g_i^eq(p0, rho(phi0), u0), h_i = h_i^eq(phi0, mu0, u0).
 *   walls      halfway bounce-back between row ny-1 and a wall, and below row 0; stencil ghosts
 *              mirror the first fluid row (zero normal gradient).
 *   clamp      optional: phi clamped to [0,1] only where rho(phi) and nu(phi) are evaluated;
 *              grad rho = (rho_A - rho_B) grad phi in every case.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- D2Q9 lattice (Sec. 2.2, listed after eq. 25): order of the printed velocity matrix ---- */
#define NQ 9
static const int ORC_CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int ORC_CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double ORC_W[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double ORC_CS2 = 1.0 / 3.0; /* c_s^2 = c^2 / 3 with c = dx/dt = 1 */
static const double ORC_RHO0 = 1.0;      /* constant rho~ = rho_0 of eq. (33) */
#define ORC_DIM 2

/* opposite direction: the index j with c_j = -c_i, found by search rather than tabulated */
static int orc_opposite(int i) {
    for (int j = 0; j < NQ; ++j)
        if (ORC_CX[j] == -ORC_CX[i] && ORC_CY[j] == -ORC_CY[i]) return j;
    return -1;
}

typedef struct {
    int32_t nx, ny;
    int32_t variant;     /* 0: quasi-incompressible, S1 = -gamma div(M grad mu); 1: incompressible, S1 = 0 */
    int32_t pscheme;     /* 0: eq.(28) with G0 of eq.(34); 1: eq.(28) with the simplified G0; 2: eq.(29) */
    int32_t fsurf;       /* 0: F_s = mu grad(phi) (Sec. 3.1); 1: F_s = -phi grad(mu) (Sec. 4.2) */
    int32_t visc;        /* 0: inverse-linear 1/nu (after eq. 17); 1: step in dynamic viscosity (Sec. 4.3) */
    int32_t bc;          /* 0: fully periodic; 1: periodic in x, halfway bounce-back walls in y */
    int32_t clamp_props; /* 1: clamp phi to [0,1] where rho(phi) and nu(phi) are evaluated */
    double rho_A, rho_B; /* densities of phase A (phi = 1) and phase B (phi = 0), eq. (3aa) */
    double nu_A, nu_B;   /* kinematic viscosities of the two phases */
    double sigma, W;     /* surface tension and interface width, eqs. (6)-(7) */
    double M_phi;        /* mobility, eq. (17) */
    double tau_h;        /* phase-field relaxation time, eq. (10) */
    double force_x, force_y; /* constant body force density (Sec. 4.3 pressure-gradient force) */
    double gravity;      /* buoyancy F_y = -(rho - rho_A) g (Sec. 4.4) */
} orc_params;

typedef struct {
    orc_params P;
    double beta, kappa, eta, gamma;
    int64_t step;
    size_t n;
    double *g, *h;           /* [NQ][ny][nx] populations at the current time (after streaming) */
    double *phiu_prev;       /* [2][ny][nx] (phi u) at the previous time, for eq. (14) */
    double *p_prev;          /* [ny][nx] pressure at the previous time (grad p reading) */
    /* per-step macroscopic work arrays */
    double *phi, *rho, *mu, *gphix, *gphiy, *lphi, *gmux, *gmuy, *lmu, *gpx, *gpy;
    double *ux, *uy, *Fx, *Fy, *S, *S1, *p, *taug, *G; /* G: [NQ][ny][nx] */
    double *gs, *hs;         /* post-collision populations */
} orc_state;

/* ------------------------------------------------------------------------------------------ */
/* Closure relations                                                                          */
/* ------------------------------------------------------------------------------------------ */

/* eqs. (6)-(7): W = sqrt(8 kappa / beta), sigma = sqrt(2 kappa beta) / 6, solved for beta, kappa */
void orc_free_energy_coeffs(double sigma, double W, double* beta, double* kappa) {
    /* kappa / beta = W^2 / 8 and kappa * beta = 18 sigma^2 */
    double kb = 18.0 * sigma * sigma;
    double k_over_b = W * W / 8.0;
    *kappa = sqrt(kb * k_over_b);
    *beta = sqrt(kb / k_over_b);
}

/* eq. (17): M_phi = eta c_s^2 (tau_h - 1/2) dt, solved for eta */
double orc_eta(double M_phi, double tau_h) { return M_phi / (ORC_CS2 * (tau_h - 0.5)); }

/* Sec. 3.2.1: gamma = (rho_A - rho_B) / (phi_A rho_B - phi_B rho_A) with phi_A = 1, phi_B = 0 */
double orc_gamma(double rho_A, double rho_B) {
    const double phi_A = 1.0, phi_B = 0.0;
    return (rho_A - rho_B) / (phi_A * rho_B - phi_B * rho_A);
}

static double orc_clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* eq. (3aa): (rho - rho_B) / (rho_A - rho_B) = (phi - phi_B) / (phi_A - phi_B) */
double orc_density(const orc_params* P, double phi) {
    const double phi_A = 1.0, phi_B = 0.0;
    double ph = P->clamp_props ? orc_clamp01(phi) : phi;
    return P->rho_B + (P->rho_A - P->rho_B) * (ph - phi_B) / (phi_A - phi_B);
}

/* kinematic viscosity: inverse-linear form after eq. (17), or the step form of Sec. 4.3 in the
 * dynamic viscosity mu = rho nu (so nu = mu / rho with rho from eq. 3aa) */
double orc_viscosity(const orc_params* P, double phi) {
    const double phi_A = 1.0, phi_B = 0.0;
    double ph = P->clamp_props ? orc_clamp01(phi) : phi;
    if (P->visc == 0) {
        double inv = (ph - phi_B) / (phi_A - phi_B) * (1.0 / P->nu_A - 1.0 / P->nu_B) + 1.0 / P->nu_B;
        return 1.0 / inv;
    }
    double mu_dyn = (phi >= 0.5) ? P->rho_A * P->nu_A : P->rho_B * P->nu_B;
    return mu_dyn / orc_density(P, phi);
}

/* nu = c_s^2 (tau_g - 1/2) dt, solved for tau_g */
double orc_tau_g(const orc_params* P, double phi) { return orc_viscosity(P, phi) / ORC_CS2 + 0.5; }

/* eq. (8): mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi) */
double orc_chemical_potential(double beta, double kappa, double phi, double lap_phi) {
    return 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap_phi;
}

/* ------------------------------------------------------------------------------------------ */
/* Isotropic finite differences, eqs. (30a)-(30b)                                              */
/* ------------------------------------------------------------------------------------------ */

/* value of a grid field at node (i + di, j + dj): periodic in x; in y periodic (bc 0) or the
 * mirrored first fluid row beyond a wall (bc 1) */
static double orc_field_at(const orc_params* P, const double* z, int i, int j) {
    int nx = P->nx, ny = P->ny;
    i = ((i % nx) + nx) % nx;
    if (P->bc == 0) {
        j = ((j % ny) + ny) % ny;
    } else {
        if (j < 0) j = -1 - j;        /* mirror about the wall half a cell below row 0 */
        if (j >= ny) j = 2 * ny - 1 - j; /* mirror about the wall half a cell above row ny-1 */
    }
    return z[(size_t)j * nx + i];
}

/* eq. (30a): grad z = sum_{i != 0} w_i c_i z(x + c_i) / c_s^2 */
void orc_gradient(const orc_params* P, const double* z, double* gx, double* gy) {
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int q = 1; q < NQ; ++q) {
                double zn = orc_field_at(P, z, i + ORC_CX[q], j + ORC_CY[q]);
                sx += ORC_W[q] * ORC_CX[q] * zn;
                sy += ORC_W[q] * ORC_CY[q] * zn;
            }
            gx[(size_t)j * P->nx + i] = sx / ORC_CS2;
            gy[(size_t)j * P->nx + i] = sy / ORC_CS2;
        }
}

/* eq. (30b): lap z = sum_{i != 0} 2 w_i [z(x + c_i) - z(x)] / c_s^2 */
void orc_laplacian(const orc_params* P, const double* z, double* lap) {
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            double zc = z[(size_t)j * P->nx + i];
            double s = 0.0;
            for (int q = 1; q < NQ; ++q)
                s += 2.0 * ORC_W[q] * (orc_field_at(P, z, i + ORC_CX[q], j + ORC_CY[q]) - zc);
            lap[(size_t)j * P->nx + i] = s / ORC_CS2;
        }
}

/* ------------------------------------------------------------------------------------------ */
/* Equilibria, force and source distributions                                                 */
/* ------------------------------------------------------------------------------------------ */

/* s_i(u) of eq. (25) */
static double orc_s(int i, double ux, double uy) {
    double cu = ORC_CX[i] * ux + ORC_CY[i] * uy;
    double uu = ux * ux + uy * uy;
    return ORC_W[i] * (cu / ORC_CS2 + cu * cu / (2.0 * ORC_CS2 * ORC_CS2) - uu / (2.0 * ORC_CS2));
}

/* eq. (33): g_0^eq = rho_0 + p/c_s^2 (w_0 - 1) + rho s_0(u); g_i^eq = p/c_s^2 w_i + rho s_i(u) */
void orc_equilibrium_g(double p, double rho, double ux, double uy, double out[NQ]) {
    for (int i = 0; i < NQ; ++i) {
        if (i == 0)
            out[i] = ORC_RHO0 + p / ORC_CS2 * (ORC_W[0] - 1.0) + rho * orc_s(0, ux, uy);
        else
            out[i] = p / ORC_CS2 * ORC_W[i] + rho * orc_s(i, ux, uy);
    }
}

/* eq. (11): h_0^eq = phi + (w_0 - 1) eta mu; h_i^eq = w_i eta mu + w_i c_i.(phi u) / c_s^2 */
void orc_equilibrium_h(double phi, double mu, double eta, double ux, double uy, double out[NQ]) {
    for (int i = 0; i < NQ; ++i) {
        if (i == 0)
            out[i] = phi + (ORC_W[0] - 1.0) * eta * mu;
        else
            out[i] = ORC_W[i] * eta * mu
                   + ORC_W[i] * (ORC_CX[i] * phi * ux + ORC_CY[i] * phi * uy) / ORC_CS2;
    }
}

/* eq. (34), written as the tensor contraction it is printed as:
 *   G_i = w_i [ u.grad(rho) + rho S1 + c_i.F / c_s^2
 *               + (c_i c_i - c_s^2 I) : (u F~ + F~ u + (2/d) rho c_s^2 S1 I) / (2 c_s^4) ]
 * The caller passes S = u.grad(rho) + rho S1 (Sec. 3.1) and F~ = F - grad(p - rho c_s^2). */
void orc_force_distribution(double rho, double ux, double uy, double Fx, double Fy, double Ftx,
                            double Fty, double S, double S1, double out[NQ]) {
    double u[2] = {ux, uy}, Ft[2] = {Ftx, Fty};
    double A[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            A[a][b] = u[a] * Ft[b] + Ft[a] * u[b]
                    + (a == b ? (2.0 / ORC_DIM) * rho * ORC_CS2 * S1 : 0.0);
    for (int i = 0; i < NQ; ++i) {
        double c[2] = {(double)ORC_CX[i], (double)ORC_CY[i]};
        double contraction = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                contraction += (c[a] * c[b] - (a == b ? ORC_CS2 : 0.0)) * A[a][b];
        double cF = c[0] * Fx + c[1] * Fy;
        out[i] = ORC_W[i] * (S + cF / ORC_CS2 + contraction / (2.0 * ORC_CS2 * ORC_CS2));
    }
}

/* simplified G_0 as printed after eq. (34) (last line of that derivation):
 *   G_0 = w_0 { (1 - 1/d) rho S1 - u.(F - grad p) / c_s^2 } */
double orc_G0_simplified(double rho, double ux, double uy, double Fx, double Fy, double gpx,
                         double gpy, double S1) {
    return ORC_W[0] * ((1.0 - 1.0 / ORC_DIM) * rho * S1
                       - (ux * (Fx - gpx) + uy * (Fy - gpy)) / ORC_CS2);
}

/* eq. (14) with the first-order difference below it (dt = 1, tau = tau_h):
 *   R_i = (1 - 1/(2 tau_h)) w_i c_i.[(phi u)^n - (phi u)^{n-1}] / c_s^2 */
void orc_source_R(double tau_h, double phiux, double phiuy, double phiux_prev, double phiuy_prev,
                  double out[NQ]) {
    double dx = phiux - phiux_prev, dy = phiuy - phiuy_prev;
    for (int i = 0; i < NQ; ++i)
        out[i] = (1.0 - 1.0 / (2.0 * tau_h)) * ORC_W[i] * (ORC_CX[i] * dx + ORC_CY[i] * dy) / ORC_CS2;
}

/* eq. (28): p = c_s^2/(1 - w_0) [ sum_{i!=0} g_i + S/2 + rho s_0(u) + (tau_g - 1/2) G_0 ];
 * eq. (29) is the same without the last term (pass with_G0 = 0) */
double orc_pressure(const double g[NQ], double S, double rho, double ux, double uy, double tau_g,
                    double G0, int with_G0) {
    double sum = 0.0;
    for (int i = 1; i < NQ; ++i) sum += g[i];
    double bracket = sum + 0.5 * S + rho * orc_s(0, ux, uy);
    if (with_G0) bracket += (tau_g - 0.5) * G0;
    return ORC_CS2 / (1.0 - ORC_W[0]) * bracket;
}

/* ------------------------------------------------------------------------------------------ */
/* Grid state                                                                                 */
/* ------------------------------------------------------------------------------------------ */

static double* orc_alloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

int orc_params_valid(const orc_params* P) {
    if (P->nx < 3 || P->ny < 3) return 0;
    if (!(P->tau_h > 0.5) || !(P->nu_A > 0.0) || !(P->nu_B > 0.0)) return 0;
    if (!(P->rho_A > 0.0) || !(P->rho_B > 0.0) || !(P->W > 0.0) || P->sigma < 0.0) return 0;
    if (P->bc != 0 && P->bc != 1) return 0;
    return 1;
}

orc_state* orc_create(const orc_params* P) {
    if (!orc_params_valid(P)) return NULL;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->P = *P;
    s->n = (size_t)P->nx * P->ny;
    orc_free_energy_coeffs(P->sigma, P->W, &s->beta, &s->kappa);
    s->eta = orc_eta(P->M_phi, P->tau_h);
    s->gamma = orc_gamma(P->rho_A, P->rho_B);
    size_t n = s->n;
    s->g = orc_alloc(NQ * n); s->h = orc_alloc(NQ * n);
    s->gs = orc_alloc(NQ * n); s->hs = orc_alloc(NQ * n); s->G = orc_alloc(NQ * n);
    s->phiu_prev = orc_alloc(2 * n); s->p_prev = orc_alloc(n);
    double** arrs[] = {&s->phi, &s->rho, &s->mu, &s->gphix, &s->gphiy, &s->lphi, &s->gmux,
                       &s->gmuy, &s->lmu, &s->gpx, &s->gpy, &s->ux, &s->uy, &s->Fx, &s->Fy,
                       &s->S, &s->S1, &s->p, &s->taug};
    for (size_t k = 0; k < sizeof(arrs) / sizeof(arrs[0]); ++k) *arrs[k] = orc_alloc(n);
    return s;
}

void orc_destroy(orc_state* s) {
    if (!s) return;
    double* arrs[] = {s->g, s->h, s->gs, s->hs, s->G, s->phiu_prev, s->p_prev, s->phi, s->rho,
                      s->mu, s->gphix, s->gphiy, s->lphi, s->gmux, s->gmuy, s->lmu, s->gpx,
                      s->gpy, s->ux, s->uy, s->Fx, s->Fy, s->S, s->S1, s->p, s->taug};
    for (size_t k = 0; k < sizeof(arrs) / sizeof(arrs[0]); ++k) free(arrs[k]);
    free(s);
}

/* Initial state (the paper gives none): u0 and p0 default to zero, mu0 from phi0 by eq. (8)
 * with the stencil of eq. (30b), h = h^eq(phi0, mu0, u0) (eq. 11), g = g^eq(p0, rho(phi0), u0)
 * (eq. 33), (phi u) before the first step = phi0 u0, p before the first step = p0. */
int orc_init(orc_state* s, const double* phi0, const double* ux0, const double* uy0,
             const double* p0) {
    size_t n = s->n;
    for (size_t k = 0; k < n; ++k) s->phi[k] = phi0[k];
    orc_laplacian(&s->P, s->phi, s->lphi);
    for (size_t k = 0; k < n; ++k) {
        double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0, p = p0 ? p0[k] : 0.0;
        double phi = phi0[k];
        double mu = orc_chemical_potential(s->beta, s->kappa, phi, s->lphi[k]);
        double heq[NQ], geq[NQ];
        orc_equilibrium_h(phi, mu, s->eta, ux, uy, heq);
        orc_equilibrium_g(p, orc_density(&s->P, phi), ux, uy, geq);
        for (int i = 0; i < NQ; ++i) {
            s->h[i * n + k] = heq[i];
            s->g[i * n + k] = geq[i];
        }
        s->phiu_prev[k] = phi * ux;
        s->phiu_prev[n + k] = phi * uy;
        s->p_prev[k] = p;
    }
    s->step = 0;
    return 0;
}

/* Macroscopic quantities of the current state, in the order the method needs them:
 * phi (eq. 18), rho (eq. 3aa), lap phi and mu (eqs. 30b, 8), grad phi, grad mu, lap mu
 * (eqs. 30a-b), F = F_s + body forces, u (eq. 27a), S1 and S (Secs. 3.1, 3.2.1),
 * grad p of the previous step, F~, G_i (eq. 34), tau_g(phi), p (eq. 28 / 29). */
static void orc_macroscopics(orc_state* s) {
    const orc_params* P = &s->P;
    size_t n = s->n;
    for (size_t k = 0; k < n; ++k) {
        double phi = 0.0;
        for (int i = 0; i < NQ; ++i) phi += s->h[i * n + k];
        s->phi[k] = phi;
        s->rho[k] = orc_density(P, phi);
    }
    orc_laplacian(P, s->phi, s->lphi);
    for (size_t k = 0; k < n; ++k)
        s->mu[k] = orc_chemical_potential(s->beta, s->kappa, s->phi[k], s->lphi[k]);
    orc_gradient(P, s->phi, s->gphix, s->gphiy);
    orc_gradient(P, s->mu, s->gmux, s->gmuy);
    orc_laplacian(P, s->mu, s->lmu);
    orc_gradient(P, s->p_prev, s->gpx, s->gpy);
    const double drho = P->rho_A - P->rho_B; /* d rho / d phi from eq. (3aa) */
    for (size_t k = 0; k < n; ++k) {
        double phi = s->phi[k], rho = s->rho[k];
        double Fsx, Fsy;
        if (P->fsurf == 0) { Fsx = s->mu[k] * s->gphix[k]; Fsy = s->mu[k] * s->gphiy[k]; }
        else { Fsx = -phi * s->gmux[k]; Fsy = -phi * s->gmuy[k]; }
        double Fx = Fsx + P->force_x;
        double Fy = Fsy + P->force_y - (rho - P->rho_A) * P->gravity;
        double mx = 0.0, my = 0.0;
        for (int i = 0; i < NQ; ++i) {
            mx += ORC_CX[i] * s->g[i * n + k];
            my += ORC_CY[i] * s->g[i * n + k];
        }
        double ux = (mx + 0.5 * Fx) / rho, uy = (my + 0.5 * Fy) / rho;
        double S1 = (P->variant == 0) ? -s->gamma * P->M_phi * s->lmu[k] : 0.0;
        double grx = drho * s->gphix[k], gry = drho * s->gphiy[k];
        double S = ux * grx + uy * gry + rho * S1;
        double Ftx = Fx - s->gpx[k] + ORC_CS2 * grx;
        double Fty = Fy - s->gpy[k] + ORC_CS2 * gry;
        double G[NQ];
        orc_force_distribution(rho, ux, uy, Fx, Fy, Ftx, Fty, S, S1, G);
        double taug = orc_tau_g(P, phi);
        double gk[NQ];
        for (int i = 0; i < NQ; ++i) gk[i] = s->g[i * n + k];
        double G0 = G[0];
        if (P->pscheme == 1) G0 = orc_G0_simplified(rho, ux, uy, Fx, Fy, s->gpx[k], s->gpy[k], S1);
        double p = orc_pressure(gk, S, rho, ux, uy, taug, G0, P->pscheme != 2);
        s->Fx[k] = Fx; s->Fy[k] = Fy; s->ux[k] = ux; s->uy[k] = uy;
        s->S1[k] = S1; s->S[k] = S; s->taug[k] = taug; s->p[k] = p;
        for (int i = 0; i < NQ; ++i) s->G[i * n + k] = G[i];
    }
}

/* One time step: macroscopics, collision of eq. (24) and eq. (10), streaming with periodic
 * wrap or halfway bounce-back, then the history (phi u) and p are kept for the next step. */
static void orc_one_step(orc_state* s) {
    const orc_params* P = &s->P;
    size_t n = s->n;
    int nx = P->nx, ny = P->ny;
    orc_macroscopics(s);
    for (size_t k = 0; k < n; ++k) {
        double geq[NQ], heq[NQ], R[NQ];
        double phi = s->phi[k], ux = s->ux[k], uy = s->uy[k];
        orc_equilibrium_g(s->p[k], s->rho[k], ux, uy, geq);
        orc_equilibrium_h(phi, s->mu[k], s->eta, ux, uy, heq);
        orc_source_R(P->tau_h, phi * ux, phi * uy, s->phiu_prev[k], s->phiu_prev[n + k], R);
        double tg = s->taug[k], th = P->tau_h;
        for (int i = 0; i < NQ; ++i) {
            double gi = s->g[i * n + k], hi = s->h[i * n + k];
            /* eq. (24), dt = 1 */
            s->gs[i * n + k] = gi - (gi - geq[i]) / tg + (1.0 - 1.0 / (2.0 * tg)) * s->G[i * n + k];
            /* eq. (10), dt = 1 */
            s->hs[i * n + k] = hi - (hi - heq[i]) / th + R[i];
        }
    }
    /* streaming: population i leaves x and arrives at x + c_i; a link that crosses a wall
     * returns the population to x in the opposite direction (halfway bounce-back, Sec. 4.3) */
    for (int j = 0; j < ny; ++j)
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)j * nx + x;
            for (int i = 0; i < NQ; ++i) {
                int xd = x + ORC_CX[i], jd = j + ORC_CY[i];
                xd = ((xd % nx) + nx) % nx;
                size_t dst;
                int idir = i;
                if (P->bc == 0) {
                    jd = ((jd % ny) + ny) % ny;
                    dst = (size_t)jd * nx + xd;
                } else if (jd < 0 || jd >= ny) {
                    idir = orc_opposite(i);
                    dst = k;
                } else {
                    dst = (size_t)jd * nx + xd;
                }
                s->g[idir * n + dst] = s->gs[i * n + k];
                s->h[idir * n + dst] = s->hs[i * n + k];
            }
        }
    for (size_t k = 0; k < n; ++k) {
        s->phiu_prev[k] = s->phi[k] * s->ux[k];
        s->phiu_prev[n + k] = s->phi[k] * s->uy[k];
        s->p_prev[k] = s->p[k];
    }
    s->step += 1;
}

void orc_step(orc_state* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) orc_one_step(s);
}

int64_t orc_step_count(const orc_state* s) { return s->step; }

/* Fields of the current state: 0 phi, 1 rho, 2 u_x, 3 u_y, 4 p (eq. 28/29 evaluated on the
 * current state), 5 mu, 6 lap phi, 7 grad phi x, 8 grad phi y, 9 S (mass source),
 * 10 F_x, 11 F_y, 12 tau_g */
int orc_read(orc_state* s, int field, double* out) {
    orc_macroscopics(s);
    double* src[] = {s->phi, s->rho, s->ux, s->uy, s->p, s->mu, s->lphi, s->gphix, s->gphiy,
                     s->S, s->Fx, s->Fy, s->taug};
    if (field < 0 || field >= (int)(sizeof(src) / sizeof(src[0]))) return -1;
    memcpy(out, src[field], s->n * sizeof(double));
    return 0;
}

/* force distribution G_i of the current state, [NQ][ny][nx] */
void orc_read_force_distribution(orc_state* s, double* out) {
    orc_macroscopics(s);
    memcpy(out, s->G, NQ * s->n * sizeof(double));
}

/* raw state: g, h ([NQ][ny][nx] each), (phi u)^{n-1} ([2][ny][nx]), p^{n-1} ([ny][nx]) */
void orc_get_state(const orc_state* s, double* g, double* h, double* phiu_prev, double* p_prev) {
    size_t n = s->n;
    if (g) memcpy(g, s->g, NQ * n * sizeof(double));
    if (h) memcpy(h, s->h, NQ * n * sizeof(double));
    if (phiu_prev) memcpy(phiu_prev, s->phiu_prev, 2 * n * sizeof(double));
    if (p_prev) memcpy(p_prev, s->p_prev, n * sizeof(double));
}

void orc_set_state(orc_state* s, const double* g, const double* h, const double* phiu_prev,
                   const double* p_prev) {
    size_t n = s->n;
    if (g) memcpy(s->g, g, NQ * n * sizeof(double));
    if (h) memcpy(s->h, h, NQ * n * sizeof(double));
    if (phiu_prev) memcpy(s->phiu_prev, phiu_prev, 2 * n * sizeof(double));
    if (p_prev) memcpy(s->p_prev, p_prev, n * sizeof(double));
}

/* global order parameter sum_x sum_i h_i(x), the quantity the scheme conserves (Sec. 3.2.2) */
double orc_sum_phi(const orc_state* s) {
    double acc = 0.0;
    for (size_t k = 0; k < NQ * s->n; ++k) acc += s->h[k];
    return acc;
}

/* Sec. 4.2: P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p with p0 = phi psi' - psi
 * and psi = beta phi^2 (phi - 1)^2 (eq. 5) */
void orc_laplace_pressure(orc_state* s, double* out) {
    orc_macroscopics(s);
    for (size_t k = 0; k < s->n; ++k) {
        double phi = s->phi[k];
        double psi = s->beta * phi * phi * (phi - 1.0) * (phi - 1.0);
        double dpsi = 4.0 * s->beta * phi * (phi - 1.0) * (phi - 0.5);
        double p0 = phi * dpsi - psi;
        double g2 = s->gphix[k] * s->gphix[k] + s->gphiy[k] * s->gphiy[k];
        out[k] = p0 - s->kappa * phi * s->lphi[k] + 0.5 * s->kappa * g2 + s->p[k];
    }
}

void orc_derived(const orc_state* s, double* out4) {
    out4[0] = s->beta; out4[1] = s->kappa; out4[2] = s->eta; out4[3] = s->gamma;
}
