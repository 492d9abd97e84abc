/*
 * FP64 CPU oracle of the phase-field lattice Boltzmann model of arXiv:1902.08933 (Yuan, Chai,
 * Wang & Shi) on the D3Q15 lattice: the three-dimensional form of the method of Sec. 3.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library. It shares no source, header, table or helper with the HIP
 * library. It is written from the paper alone, in plain loops, in double precision, in the
 * order in which the paper states the method.
 *
 * Paper map (section / equation labels as printed in the paper):
 *   lattice                 Sec. 2.2, D3Q15 weights and velocity matrix (after eq. 25)
 *   hydrodynamic LB         eq. (24) evolution, eq. (33) equilibrium, eq. (34) force term with
 *                           d = 3, eq. (27a) velocity, eq. (28) / (29) pressure
 *   phase-field LB          eq. (10) evolution, eq. (11) equilibrium, eq. (14) source,
 *                           eq. (18) order parameter, eq. (17) mobility
 *   closure                 eq. (3aa) density, eq. (8) chemical potential, eqs. (6)-(7), Sec. 3.1
 *                           surface tension and S = u.grad(rho) + rho S1, Sec. 3.2.1 gamma
 *   stencils                eqs. (30a), (30b) over the D3Q15 neighbours
 *   Laplace diagnostic      Sec. 4.2, P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p
 *
 * The d-independent closure relations (eqs. 6-8, 17 and gamma) are the two-dimensional
 * oracle's functions, linked from the same library.
 *
 * Readings (the paper gives the lattice but no three-dimensional case):
 *   d          the trace term (2/d) rho c_s^2 S1 I of eq. (34) and the simplified G_0 printed
 *              after it use d = 3.
 *   walls      halfway bounce-back half a cell below plane z = 0 and above plane z = nz - 1
 *              (bc 1); x and y are periodic. Stencil ghosts beyond a wall mirror the first fluid
 *              plane. The buoyancy force acts along -z: F_z = -(rho - rho_A) g.
 *   the rest   as in the two-dimensional oracle: G_0 of eq. (34) at i = 0 in eq. (28)
 *              (pscheme 0), grad p of the previous step, R_i with tau_h, (phi u) and p before
 *              the first step taken from the initial fields, equilibrium initial populations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- D3Q15 (Sec. 2.2): columns of the printed velocity matrix, in order ---- */
#define Q3 15
static const int O3_C[Q3][3] = {
    {0, 0, 0},  {1, 0, 0},   {0, 1, 0},  {0, 0, 1},  {-1, 0, 0},  {0, -1, 0},   {0, 0, -1},
    {1, 1, 1},  {1, 1, -1},  {1, -1, 1}, {-1, 1, 1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1},
    {1, -1, -1}};
static double o3_w(int i) { return i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0); }
static const double O3_CS2 = 1.0 / 3.0;
static const double O3_RHO0 = 1.0; /* constant rho~ = rho_0 of eq. (33) */
#define O3_DIM 3

/* closure relations of the two-dimensional oracle (independent of the lattice) */
void orc_free_energy_coeffs(double sigma, double W, double* beta, double* kappa);
double orc_eta(double M_phi, double tau_h);
double orc_gamma(double rho_A, double rho_B);
double orc_chemical_potential(double beta, double kappa, double phi, double lap_phi);

static int o3_opposite(int i) {
    for (int j = 0; j < Q3; ++j)
        if (O3_C[j][0] == -O3_C[i][0] && O3_C[j][1] == -O3_C[i][1] && O3_C[j][2] == -O3_C[i][2])
            return j;
    return -1;
}

/* velocities and weights as the oracle holds them (for the lattice pins) */
void o3_lattice(int32_t* c, double* w) {
    for (int i = 0; i < Q3; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = O3_C[i][a];
        w[i] = o3_w(i);
    }
}

typedef struct {
    int32_t nx, ny, nz;
    int32_t variant;     /* 0 quasi-incompressible, 1 incompressible */
    int32_t pscheme;     /* 0 eq.(28) with G0 of eq.(34); 1 the simplified G0; 2 eq.(29) */
    int32_t fsurf;       /* 0 mu grad phi; 1 -phi grad mu */
    int32_t visc;        /* 0 inverse-linear; 1 step in the dynamic viscosity */
    int32_t bc;          /* 0 periodic; 1 walls in z */
    int32_t clamp_props;
    int32_t pad;
    double rho_A, rho_B, nu_A, nu_B, sigma, W, M_phi, tau_h;
    double force_x, force_y, force_z, gravity;
} o3_params;

typedef struct {
    o3_params P;
    double beta, kappa, eta, gamma;
    int64_t step;
    size_t n;
    double *g, *h, *gs, *hs, *G;   /* [Q3][nz][ny][nx] */
    double *phiu_prev;             /* [3][nz][ny][nx] */
    double *p_prev;
    double *phi, *rho, *mu, *lphi, *lmu, *p, *taug, *S, *S1;
    double *gphi[3], *gmu[3], *gp[3], *u[3], *F[3];
} o3_state;

static double o3_clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* eq. (3aa) with phi_A = 1, phi_B = 0 */
double o3_density(const o3_params* P, double phi) {
    double ph = P->clamp_props ? o3_clamp01(phi) : phi;
    return P->rho_B + (P->rho_A - P->rho_B) * ph;
}

/* inverse-linear 1/nu (after eq. 17), or the step in the dynamic viscosity (Sec. 4.3) */
double o3_viscosity(const o3_params* P, double phi) {
    double ph = P->clamp_props ? o3_clamp01(phi) : phi;
    if (P->visc == 0) return 1.0 / (ph * (1.0 / P->nu_A - 1.0 / P->nu_B) + 1.0 / P->nu_B);
    double mu_dyn = (phi >= 0.5) ? P->rho_A * P->nu_A : P->rho_B * P->nu_B;
    return mu_dyn / o3_density(P, phi);
}

/* ---- stencils, eqs. (30a)-(30b) ---- */

/* value at node (x, y, z): periodic in x and y; in z periodic (bc 0) or the mirrored first
 * fluid plane beyond a wall (bc 1) */
static double o3_field_at(const o3_params* P, const double* f, int x, int y, int z) {
    int nx = P->nx, ny = P->ny, nz = P->nz;
    x = ((x % nx) + nx) % nx;
    y = ((y % ny) + ny) % ny;
    if (P->bc == 0) {
        z = ((z % nz) + nz) % nz;
    } else {
        if (z < 0) z = -1 - z;
        if (z >= nz) z = 2 * nz - 1 - z;
    }
    return f[((size_t)z * ny + y) * nx + x];
}

void o3_gradient(const o3_params* P, const double* f, double* gx, double* gy, double* gz) {
    double* out[3] = {gx, gy, gz};
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                double s[3] = {0.0, 0.0, 0.0};
                for (int i = 1; i < Q3; ++i) {
                    double fn = o3_field_at(P, f, x + O3_C[i][0], y + O3_C[i][1], z + O3_C[i][2]);
                    for (int a = 0; a < 3; ++a) s[a] += o3_w(i) * O3_C[i][a] * fn;
                }
                size_t k = ((size_t)z * P->ny + y) * P->nx + x;
                for (int a = 0; a < 3; ++a) out[a][k] = s[a] / O3_CS2;
            }
}

void o3_laplacian(const o3_params* P, const double* f, double* lap) {
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                size_t k = ((size_t)z * P->ny + y) * P->nx + x;
                double s = 0.0;
                for (int i = 1; i < Q3; ++i)
                    s += 2.0 * o3_w(i) *
                         (o3_field_at(P, f, x + O3_C[i][0], y + O3_C[i][1], z + O3_C[i][2]) - f[k]);
                lap[k] = s / O3_CS2;
            }
}

/* ---- equilibria, force and source distributions ---- */

static double o3_cdot(int i, const double* v) {
    return O3_C[i][0] * v[0] + O3_C[i][1] * v[1] + O3_C[i][2] * v[2];
}

/* s_i(u) of eq. (25) */
static double o3_s(int i, const double* u) {
    double cu = o3_cdot(i, u), uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return o3_w(i) * (cu / O3_CS2 + cu * cu / (2.0 * O3_CS2 * O3_CS2) - uu / (2.0 * O3_CS2));
}

/* eq. (33) */
void o3_equilibrium_g(double p, double rho, const double* u, double* out) {
    for (int i = 0; i < Q3; ++i)
        out[i] = (i == 0 ? O3_RHO0 + p / O3_CS2 * (o3_w(0) - 1.0) : p / O3_CS2 * o3_w(i))
               + rho * o3_s(i, u);
}

/* eq. (11) */
void o3_equilibrium_h(double phi, double mu, double eta, const double* u, double* out) {
    double pu[3] = {phi * u[0], phi * u[1], phi * u[2]};
    for (int i = 0; i < Q3; ++i)
        out[i] = (i == 0) ? phi + (o3_w(0) - 1.0) * eta * mu
                          : o3_w(i) * eta * mu + o3_w(i) * o3_cdot(i, pu) / O3_CS2;
}

/* eq. (34) as the tensor contraction it is printed as, d = 3:
 *   G_i = w_i [ S + c_i.F / c_s^2 + (c_i c_i - c_s^2 I) : (u F~ + F~ u + (2/d) rho c_s^2 S1 I)
 *               / (2 c_s^4) ] */
void o3_force_distribution(double rho, const double* u, const double* F, const double* Ft,
                           double S, double S1, double* out) {
    double A[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            A[a][b] = u[a] * Ft[b] + Ft[a] * u[b]
                    + (a == b ? (2.0 / O3_DIM) * rho * O3_CS2 * S1 : 0.0);
    for (int i = 0; i < Q3; ++i) {
        double contraction = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                contraction += (O3_C[i][a] * O3_C[i][b] - (a == b ? O3_CS2 : 0.0)) * A[a][b];
        out[i] = o3_w(i) * (S + o3_cdot(i, F) / O3_CS2 + contraction / (2.0 * O3_CS2 * O3_CS2));
    }
}

/* simplified G_0 printed after eq. (34): w_0 { (1 - 1/d) rho S1 - u.(F - grad p) / c_s^2 } */
double o3_G0_simplified(double rho, const double* u, const double* F, const double* gp, double S1) {
    double d = 0.0;
    for (int a = 0; a < 3; ++a) d += u[a] * (F[a] - gp[a]);
    return o3_w(0) * ((1.0 - 1.0 / O3_DIM) * rho * S1 - d / O3_CS2);
}

/* eq. (14) with the first-order time difference: R_i = (1 - 1/(2 tau_h)) w_i c_i.d(phi u)/c_s^2 */
void o3_source_R(double tau_h, const double* phiu, const double* phiu_prev, double* out) {
    double d[3] = {phiu[0] - phiu_prev[0], phiu[1] - phiu_prev[1], phiu[2] - phiu_prev[2]};
    for (int i = 0; i < Q3; ++i)
        out[i] = (1.0 - 1.0 / (2.0 * tau_h)) * o3_w(i) * o3_cdot(i, d) / O3_CS2;
}

/* eq. (28): p = c_s^2/(1 - w_0) [ sum_{i!=0} g_i + S/2 + rho s_0(u) + (tau_g - 1/2) G_0 ];
 * eq. (29) without the last term */
double o3_pressure(const double* g, double S, double rho, const double* u, double tau_g, double G0,
                   int with_G0) {
    double sum = 0.0;
    for (int i = 1; i < Q3; ++i) sum += g[i];
    double bracket = sum + 0.5 * S + rho * o3_s(0, u);
    if (with_G0) bracket += (tau_g - 0.5) * G0;
    return O3_CS2 / (1.0 - o3_w(0)) * bracket;
}

/* ---- grid state ---- */

int o3_params_valid(const o3_params* P) {
    if (P->nx < 3 || P->ny < 3 || P->nz < 3) return 0;
    if (!(P->tau_h > 0.5) || !(P->nu_A > 0.0) || !(P->nu_B > 0.0)) return 0;
    if (!(P->rho_A > 0.0) || !(P->rho_B > 0.0) || !(P->W > 0.0) || P->sigma < 0.0) return 0;
    if (P->bc != 0 && P->bc != 1) return 0;
    return 1;
}

static double* o3_alloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

o3_state* o3_create(const o3_params* P) {
    if (!o3_params_valid(P)) return NULL;
    o3_state* s = (o3_state*)calloc(1, sizeof(o3_state));
    s->P = *P;
    size_t n = s->n = (size_t)P->nx * P->ny * P->nz;
    orc_free_energy_coeffs(P->sigma, P->W, &s->beta, &s->kappa);
    s->eta = orc_eta(P->M_phi, P->tau_h);
    s->gamma = orc_gamma(P->rho_A, P->rho_B);
    s->g = o3_alloc(Q3 * n); s->h = o3_alloc(Q3 * n);
    s->gs = o3_alloc(Q3 * n); s->hs = o3_alloc(Q3 * n); s->G = o3_alloc(Q3 * n);
    s->phiu_prev = o3_alloc(3 * n);
    s->p_prev = o3_alloc(n); s->phi = o3_alloc(n); s->rho = o3_alloc(n); s->mu = o3_alloc(n);
    s->lphi = o3_alloc(n); s->lmu = o3_alloc(n); s->p = o3_alloc(n); s->taug = o3_alloc(n);
    s->S = o3_alloc(n); s->S1 = o3_alloc(n);
    for (int a = 0; a < 3; ++a) {
        s->gphi[a] = o3_alloc(n); s->gmu[a] = o3_alloc(n); s->gp[a] = o3_alloc(n);
        s->u[a] = o3_alloc(n); s->F[a] = o3_alloc(n);
    }
    return s;
}

void o3_destroy(o3_state* s) {
    if (!s) return;
    double* one[] = {s->g, s->h, s->gs, s->hs, s->G, s->phiu_prev, s->p_prev, s->phi, s->rho,
                     s->mu, s->lphi, s->lmu, s->p, s->taug, s->S, s->S1};
    for (size_t j = 0; j < sizeof(one) / sizeof(one[0]); ++j) free(one[j]);
    for (int a = 0; a < 3; ++a) {
        free(s->gphi[a]); free(s->gmu[a]); free(s->gp[a]); free(s->u[a]); free(s->F[a]);
    }
    free(s);
}

/* initial state: mu0 from phi0 by eq. (8) with eq. (30b), h = h^eq(phi0, mu0, u0),
 * g = g^eq(p0, rho(phi0), u0), histories from the initial fields (any of u, p may be NULL) */
int o3_init(o3_state* s, const double* phi0, const double* ux0, const double* uy0,
            const double* uz0, const double* p0) {
    size_t n = s->n;
    memcpy(s->phi, phi0, n * sizeof(double));
    o3_laplacian(&s->P, s->phi, s->lphi);
    const double* u0[3] = {ux0, uy0, uz0};
    for (size_t k = 0; k < n; ++k) {
        double u[3];
        for (int a = 0; a < 3; ++a) u[a] = u0[a] ? u0[a][k] : 0.0;
        double p = p0 ? p0[k] : 0.0, phi = phi0[k];
        double mu = orc_chemical_potential(s->beta, s->kappa, phi, s->lphi[k]);
        double heq[Q3], geq[Q3];
        o3_equilibrium_h(phi, mu, s->eta, u, heq);
        o3_equilibrium_g(p, o3_density(&s->P, phi), u, geq);
        for (int i = 0; i < Q3; ++i) {
            s->h[i * n + k] = heq[i];
            s->g[i * n + k] = geq[i];
        }
        for (int a = 0; a < 3; ++a) s->phiu_prev[a * n + k] = phi * u[a];
        s->p_prev[k] = p;
    }
    s->step = 0;
    return 0;
}

/* macroscopic quantities of the current state, in the order the method needs them (as in the
 * two-dimensional oracle) */
static void o3_macroscopics(o3_state* s) {
    const o3_params* P = &s->P;
    size_t n = s->n;
    for (size_t k = 0; k < n; ++k) {
        double phi = 0.0;
        for (int i = 0; i < Q3; ++i) phi += s->h[i * n + k];
        s->phi[k] = phi;
        s->rho[k] = o3_density(P, phi);
    }
    o3_laplacian(P, s->phi, s->lphi);
    for (size_t k = 0; k < n; ++k)
        s->mu[k] = orc_chemical_potential(s->beta, s->kappa, s->phi[k], s->lphi[k]);
    o3_gradient(P, s->phi, s->gphi[0], s->gphi[1], s->gphi[2]);
    o3_gradient(P, s->mu, s->gmu[0], s->gmu[1], s->gmu[2]);
    o3_laplacian(P, s->mu, s->lmu);
    o3_gradient(P, s->p_prev, s->gp[0], s->gp[1], s->gp[2]);
    const double drho = P->rho_A - P->rho_B;
    const double body[3] = {P->force_x, P->force_y, P->force_z};
    for (size_t k = 0; k < n; ++k) {
        double phi = s->phi[k], rho = s->rho[k];
        double F[3], u[3], Ft[3], gr[3], gp[3];
        for (int a = 0; a < 3; ++a) {
            double Fs = (P->fsurf == 0) ? s->mu[k] * s->gphi[a][k] : -phi * s->gmu[a][k];
            F[a] = Fs + body[a];
        }
        F[2] -= (rho - P->rho_A) * P->gravity;
        for (int a = 0; a < 3; ++a) {
            double m = 0.0;
            for (int i = 0; i < Q3; ++i) m += O3_C[i][a] * s->g[i * n + k];
            u[a] = (m + 0.5 * F[a]) / rho; /* eq. (27a) */
        }
        double S1 = (P->variant == 0) ? -s->gamma * P->M_phi * s->lmu[k] : 0.0;
        double S = rho * S1;
        for (int a = 0; a < 3; ++a) {
            gr[a] = drho * s->gphi[a][k];
            gp[a] = s->gp[a][k];
            S += u[a] * gr[a];
        }
        for (int a = 0; a < 3; ++a) Ft[a] = F[a] - gp[a] + O3_CS2 * gr[a];
        double G[Q3], gk[Q3];
        o3_force_distribution(rho, u, F, Ft, S, S1, G);
        double taug = o3_viscosity(P, phi) / O3_CS2 + 0.5;
        for (int i = 0; i < Q3; ++i) gk[i] = s->g[i * n + k];
        double G0 = (P->pscheme == 1) ? o3_G0_simplified(rho, u, F, gp, S1) : G[0];
        s->p[k] = o3_pressure(gk, S, rho, u, taug, G0, P->pscheme != 2);
        for (int a = 0; a < 3; ++a) { s->u[a][k] = u[a]; s->F[a][k] = F[a]; }
        s->S[k] = S; s->S1[k] = S1; s->taug[k] = taug;
        for (int i = 0; i < Q3; ++i) s->G[i * n + k] = G[i];
    }
}

/* one step: collisions of eq. (24) and eq. (10), then streaming (periodic, or halfway
 * bounce-back at the z walls), then the histories */
static void o3_one_step(o3_state* s) {
    const o3_params* P = &s->P;
    size_t n = s->n;
    int nx = P->nx, ny = P->ny, nz = P->nz;
    o3_macroscopics(s);
    for (size_t k = 0; k < n; ++k) {
        double u[3] = {s->u[0][k], s->u[1][k], s->u[2][k]}, phi = s->phi[k];
        double pu[3] = {phi * u[0], phi * u[1], phi * u[2]};
        double pp[3] = {s->phiu_prev[k], s->phiu_prev[n + k], s->phiu_prev[2 * n + k]};
        double geq[Q3], heq[Q3], R[Q3];
        o3_equilibrium_g(s->p[k], s->rho[k], u, geq);
        o3_equilibrium_h(phi, s->mu[k], s->eta, u, heq);
        o3_source_R(P->tau_h, pu, pp, R);
        double tg = s->taug[k], th = P->tau_h;
        for (int i = 0; i < Q3; ++i) {
            double gi = s->g[i * n + k], hi = s->h[i * n + k];
            s->gs[i * n + k] = gi - (gi - geq[i]) / tg + (1.0 - 1.0 / (2.0 * tg)) * s->G[i * n + k];
            s->hs[i * n + k] = hi - (hi - heq[i]) / th + R[i];
        }
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t k = ((size_t)z * ny + y) * nx + x;
                for (int i = 0; i < Q3; ++i) {
                    int xd = ((x + O3_C[i][0]) % nx + nx) % nx;
                    int yd = ((y + O3_C[i][1]) % ny + ny) % ny;
                    int zd = z + O3_C[i][2];
                    size_t dst;
                    int idir = i;
                    if (P->bc == 0) {
                        zd = ((zd % nz) + nz) % nz;
                        dst = ((size_t)zd * ny + yd) * nx + xd;
                    } else if (zd < 0 || zd >= nz) {
                        idir = o3_opposite(i);
                        dst = k;
                    } else {
                        dst = ((size_t)zd * ny + yd) * nx + xd;
                    }
                    s->g[idir * n + dst] = s->gs[i * n + k];
                    s->h[idir * n + dst] = s->hs[i * n + k];
                }
            }
    for (size_t k = 0; k < n; ++k) {
        for (int a = 0; a < 3; ++a) s->phiu_prev[a * n + k] = s->phi[k] * s->u[a][k];
        s->p_prev[k] = s->p[k];
    }
    s->step += 1;
}

void o3_step(o3_state* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) o3_one_step(s);
}

int64_t o3_step_count(const o3_state* s) { return s->step; }

/* fields: 0 phi, 1 rho, 2-4 u, 5 p, 6 mu, 7 lap phi, 8-10 grad phi, 11 S, 12-14 F, 15 tau_g */
int o3_read(o3_state* s, int field, double* out) {
    o3_macroscopics(s);
    double* src[] = {s->phi, s->rho, s->u[0], s->u[1], s->u[2], s->p, s->mu, s->lphi,
                     s->gphi[0], s->gphi[1], s->gphi[2], s->S, s->F[0], s->F[1], s->F[2], s->taug};
    if (field < 0 || field >= (int)(sizeof(src) / sizeof(src[0]))) return -1;
    memcpy(out, src[field], s->n * sizeof(double));
    return 0;
}

void o3_get_state(const o3_state* s, double* g, double* h, double* phiu_prev, double* p_prev) {
    size_t n = s->n;
    if (g) memcpy(g, s->g, Q3 * n * sizeof(double));
    if (h) memcpy(h, s->h, Q3 * n * sizeof(double));
    if (phiu_prev) memcpy(phiu_prev, s->phiu_prev, 3 * n * sizeof(double));
    if (p_prev) memcpy(p_prev, s->p_prev, n * sizeof(double));
}

void o3_set_state(o3_state* s, const double* g, const double* h, const double* phiu_prev,
                  const double* p_prev) {
    size_t n = s->n;
    if (g) memcpy(s->g, g, Q3 * n * sizeof(double));
    if (h) memcpy(s->h, h, Q3 * n * sizeof(double));
    if (phiu_prev) memcpy(s->phiu_prev, phiu_prev, 3 * n * sizeof(double));
    if (p_prev) memcpy(s->p_prev, p_prev, n * sizeof(double));
}

double o3_sum_phi(const o3_state* s) {
    double acc = 0.0;
    for (size_t k = 0; k < Q3 * s->n; ++k) acc += s->h[k];
    return acc;
}

/* Sec. 4.2 pressure P = p0 - kappa phi lap(phi) + kappa |grad phi|^2 / 2 + p */
void o3_laplace_pressure(o3_state* s, double* out) {
    o3_macroscopics(s);
    for (size_t k = 0; k < s->n; ++k) {
        double phi = s->phi[k];
        double psi = s->beta * phi * phi * (phi - 1.0) * (phi - 1.0);
        double dpsi = 4.0 * s->beta * phi * (phi - 1.0) * (phi - 0.5);
        double g2 = 0.0;
        for (int a = 0; a < 3; ++a) g2 += s->gphi[a][k] * s->gphi[a][k];
        out[k] = (phi * dpsi - psi) - s->kappa * phi * s->lphi[k] + 0.5 * s->kappa * g2 + s->p[k];
    }
}
