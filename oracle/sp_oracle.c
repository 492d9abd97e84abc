/*
 * FP64 CPU oracle of the generalized single-phase lattice Boltzmann model with a mass source
 * of Yuan, Chai, Wang & Shi (arXiv:1902.08933), Sec. 2: the evolution eq. (24), the
 * equilibrium eq. (25) and the force term eq. (27), in the two reductions the paper spells
 * out:
 *   model 0  Remark 1, nearly incompressible: rho~ = rho and p = rho c_s^2, so the equilibrium
 *            is eq. (29bb), g_i^eq = rho [w_i + s_i(u)]; rho = sum_i g_i + S/2 (eq. 27aa),
 *            u from eq. (27a); the force term's bracket is uF + Fu - uu S + Q (div u) I.
 *   model 1  Remark 3, incompressible with a mass source: rho~ = rho_0, rho = 1; the
 *            equilibrium is eq. (25) with rho = 1, u from eq. (27a), p from eq. (28) (or
 *            eq. (29)); the bracket is uF + Fu + Q S I (div u = S).
 * with Q = (2/d) rho c_s^2 - xi / (tau_g - 1/2) (after eq. 27) and tau_g from
 * nu = c_s^2 (tau_g - 1/2).
 *
 * TEST INFRASTRUCTURE, like lbpf_oracle.c: plain loops in double precision, in the order the
 * paper states the method; it shares no code with the HIP library.
 *
 * Readings (each documented where it is used):
 *   div u    model 0 needs div u in the force term at the time the force is evaluated; the
 *            divergence (eq. 30a) of the previous step's velocity is used, the initial u
 *            before the first step.
 *   full     model 0: full = 1 keeps the -uu S term as printed in Remark 1's force term,
 *            full = 0 drops it (Remark 1 notes it is O(Ma^3)). model 1: full = 1 restores the
 *            terms of eq. (27) that Remark 3 neglects: d_t(p - rho_0 c_s^2) I, the -grad p
 *            part of F~ = F - grad(p - rho c_s^2) and -uu S~ (S~ = S since rho and rho~ are
 *            constant); full = 0 is Remark 3's force term.
 *            grad p is eq. (30a) of the previous step's pressure (the initial p before the
 *            first step). d_t p is the backward difference p^n - p^{n-1} at the current
 *            level: G_0 is affine in it, so eq. (28) is solved for p^n in closed form. (A
 *            lagged difference p^{n-1} - p^{n-2} feeds back into eq. (28) and grows without
 *            bound; the current-level difference is stable.)
 *   fields   S(x) and F(x) are given per node and constant in time; with drag lambda the
 *            force is F = F_ext - lambda rho u, a force that depends on u (the case Remark 4 is
 *            written for): under eq. (24) the velocity of eq. (27a) is then implicit and, the
 *            dependence being linear, solved in closed form.
 *   Remark 4 (scheme 1, model 0 only) evolves f~ of eq. (21bb) itself with the explicit
 *            discretization of D_i G_i: rho~ = sum f~, rho u = sum c f~; G_i(x + c_i) across a
 *            wall link is G_i(x); before the first step G(t - 1) = G(t).
 *   init     g_i = g_i^eq of the initial fields.
 *   walls    halfway bounce-back below row 0 and above row ny-1 (bc 1); stencil ghosts mirror
 *            the first fluid row.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SP_NQ 9
static const int SP_CX[SP_NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int SP_CY[SP_NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double SP_W[SP_NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double SP_CS2 = 1.0 / 3.0;
#define SP_DIM 2

typedef struct {
    int32_t nx, ny;
    int32_t model;   /* 0: Remark 1 (nearly incompressible); 1: Remark 3 (incompressible + source) */
    int32_t pscheme; /* model 1: 0 eq. (28) with G_0 of the force term at i = 0, 1 eq. (29) */
    int32_t full;    /* see the header */
    int32_t bc;      /* 0 periodic; 1 periodic in x, halfway bounce-back walls in y */
    double nu;       /* kinematic viscosity */
    double xi;       /* bulk viscosity */
    double rho0;     /* model 1: the constant rho~ */
    double drag;     /* model 0: lambda >= 0, the force is F = F_ext - lambda rho u (it depends on u) */
    int32_t scheme;  /* model 0: 0 eq. (24) with g = f~ - G/2 (eq. 23a); 1 Remark 4, the
                        explicit D_i G_i scheme on f~ itself */
    int32_t pad;
} sp_params;

typedef struct {
    sp_params P;
    double tau;
    int64_t step;
    size_t n;
    double *g, *gs;              /* [NQ][ny][nx] populations after streaming / after collision */
    double *S, *Fx, *Fy;         /* source and force fields */
    double *ux_prev, *uy_prev;   /* model 0: velocity of the previous step (div u reading) */
    double *p_prev;              /* model 1: pressure of the previous step */
    double *rho, *ux, *uy, *p, *G; /* per-step work arrays; G is [NQ][ny][nx] */
    double *G_prev;              /* Remark 4: the force distribution of the previous step */
    double *w1, *w2, *w3;        /* stencil scratch */
} sp_state;

static int sp_opposite(int i) {
    for (int j = 0; j < SP_NQ; ++j)
        if (SP_CX[j] == -SP_CX[i] && SP_CY[j] == -SP_CY[i]) return j;
    return -1;
}

/* s_i(u) of eq. (25) */
static double sp_s(int i, double ux, double uy) {
    double cu = SP_CX[i] * ux + SP_CY[i] * uy;
    double uu = ux * ux + uy * uy;
    return SP_W[i] * (cu / SP_CS2 + cu * cu / (2.0 * SP_CS2 * SP_CS2) - uu / (2.0 * SP_CS2));
}

/* eq. (27): G_i = w_i { S + c_i.F / c_s^2 + (c_i c_i - c_s^2 I) : A / (2 c_s^4) } for a given
 * symmetric 2x2 bracket A = (axx, axy, ayy), contracted as printed */
void sp_force_distribution(double S, double Fx, double Fy, double axx, double axy, double ayy,
                           double out[SP_NQ]) {
    for (int i = 0; i < SP_NQ; ++i) {
        double cx = SP_CX[i], cy = SP_CY[i];
        double mxx = cx * cx - SP_CS2, mxy = cx * cy, myy = cy * cy - SP_CS2;
        double contr = mxx * axx + 2.0 * mxy * axy + myy * ayy;
        out[i] = SP_W[i] * (S + (cx * Fx + cy * Fy) / SP_CS2 + contr / (2.0 * SP_CS2 * SP_CS2));
    }
}

/* the bracket of eq. (27): d_t(p - rho~ c_s^2) I + u F~ + F~ u - u u S~ + Q (div u) I */
void sp_bracket(double dtp, double ux, double uy, double Ftx, double Fty, double St, double Q,
                double divu, double* axx, double* axy, double* ayy) {
    *axx = dtp + 2.0 * ux * Ftx - ux * ux * St + Q * divu;
    *axy = ux * Fty + Ftx * uy - ux * uy * St;
    *ayy = dtp + 2.0 * uy * Fty - uy * uy * St + Q * divu;
}

/* eq. (29bb): g_i^eq = rho [w_i + s_i(u)] (model 0) */
void sp_equilibrium_ni(double rho, double ux, double uy, double out[SP_NQ]) {
    for (int i = 0; i < SP_NQ; ++i) out[i] = rho * (SP_W[i] + sp_s(i, ux, uy));
}

/* eq. (25) with rho = 1 (model 1): g_0^eq = rho_0 + p/c_s^2 (w_0 - 1) + s_0(u),
 * g_i^eq = p/c_s^2 w_i + s_i(u) */
void sp_equilibrium_inc(double rho0, double p, double ux, double uy, double out[SP_NQ]) {
    out[0] = rho0 + p / SP_CS2 * (SP_W[0] - 1.0) + sp_s(0, ux, uy);
    for (int i = 1; i < SP_NQ; ++i) out[i] = p / SP_CS2 * SP_W[i] + sp_s(i, ux, uy);
}

/* eq. (28) with rho = 1 (scheme 0) or eq. (29) (scheme 1) */
double sp_pressure_inc(const double g[SP_NQ], double S, double ux, double uy, double tau,
                       double G0, int scheme) {
    double sum = 0.0;
    for (int i = 1; i < SP_NQ; ++i) sum += g[i];
    double br = sum + 0.5 * S + sp_s(0, ux, uy);
    if (scheme == 0) br += (tau - 0.5) * G0;
    return SP_CS2 / (1.0 - SP_W[0]) * br;
}

static double sp_at(const sp_params* P, const double* z, int i, int j) {
    int nx = P->nx, ny = P->ny;
    i = ((i % nx) + nx) % nx;
    if (P->bc == 0) {
        j = ((j % ny) + ny) % ny;
    } else {
        if (j < 0) j = -1 - j;
        if (j >= ny) j = 2 * ny - 1 - j;
    }
    return z[(size_t)j * nx + i];
}

/* eq. (30a) of a field */
static void sp_gradient(const sp_params* P, const double* z, double* gx, double* gy) {
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int q = 1; q < SP_NQ; ++q) {
                double zn = sp_at(P, z, i + SP_CX[q], j + SP_CY[q]);
                sx += SP_W[q] * SP_CX[q] * zn;
                sy += SP_W[q] * SP_CY[q] * zn;
            }
            gx[(size_t)j * P->nx + i] = sx / SP_CS2;
            gy[(size_t)j * P->nx + i] = sy / SP_CS2;
        }
}

int sp_params_valid(const sp_params* P) {
    if (P->nx < 3 || P->ny < 3) return 0;
    if (P->model != 0 && P->model != 1) return 0;
    if (!(P->nu > 0.0)) return 0;
    if (!(P->drag >= 0.0) || (P->drag != 0.0 && P->model != 0)) return 0;
    if (P->scheme != 0 && (P->scheme != 1 || P->model != 0)) return 0;
    return 1;
}

sp_state* sp_create(const sp_params* P) {
    if (!sp_params_valid(P)) return NULL;
    sp_state* s = (sp_state*)calloc(1, sizeof(sp_state));
    s->P = *P;
    s->tau = P->nu / SP_CS2 + 0.5;
    s->n = (size_t)P->nx * P->ny;
    size_t n = s->n;
    s->g = calloc(SP_NQ * n, sizeof(double));
    s->gs = calloc(SP_NQ * n, sizeof(double));
    s->G = calloc(SP_NQ * n, sizeof(double));
    s->G_prev = calloc(SP_NQ * n, sizeof(double));
    double** one[] = {&s->S, &s->Fx, &s->Fy, &s->ux_prev, &s->uy_prev, &s->p_prev,
                      &s->rho, &s->ux, &s->uy, &s->p, &s->w1, &s->w2, &s->w3};
    for (size_t k = 0; k < sizeof(one) / sizeof(one[0]); ++k) *one[k] = calloc(n, sizeof(double));
    return s;
}

void sp_destroy(sp_state* s) {
    if (!s) return;
    double* all[] = {s->g, s->gs, s->G, s->G_prev, s->S, s->Fx, s->Fy, s->ux_prev, s->uy_prev, s->p_prev,
                     s->rho, s->ux, s->uy, s->p, s->w1, s->w2, s->w3};
    for (size_t k = 0; k < sizeof(all) / sizeof(all[0]); ++k) free(all[k]);
    free(s);
}

/* Initial state: rho0 (model 0: density; model 1: pressure p), u0, and the source and force
 * fields (NULL: zero). g_i = g_i^eq of the initial fields. */
void sp_init(sp_state* s, const double* a0, const double* ux0, const double* uy0,
             const double* S, const double* Fx, const double* Fy) {
    size_t n = s->n;
    for (size_t k = 0; k < n; ++k) {
        double a = a0 ? a0[k] : (s->P.model == 0 ? 1.0 : 0.0);
        double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
        double geq[SP_NQ];
        if (s->P.model == 0) sp_equilibrium_ni(a, ux, uy, geq);
        else sp_equilibrium_inc(s->P.rho0, a, ux, uy, geq);
        for (int i = 0; i < SP_NQ; ++i) s->g[i * n + k] = geq[i];
        s->S[k] = S ? S[k] : 0.0;
        s->Fx[k] = Fx ? Fx[k] : 0.0;
        s->Fy[k] = Fy ? Fy[k] : 0.0;
        s->ux_prev[k] = ux;
        s->uy_prev[k] = uy;
        s->p_prev[k] = (s->P.model == 1) ? a : 0.0;
    }
    s->step = 0;
}

/* Macroscopic quantities and the force term of the current state. */
static void sp_macroscopics(sp_state* s) {
    const sp_params* P = &s->P;
    size_t n = s->n;
    double tau = s->tau;
    if (P->model == 0) {
        /* div u of the previous step's velocity (reading "div u") */
        sp_gradient(P, s->ux_prev, s->w1, s->w3);
        sp_gradient(P, s->uy_prev, s->w3, s->w2);
        for (size_t k = 0; k < n; ++k) {
            double g[SP_NQ], sum = 0.0, mx = 0.0, my = 0.0;
            for (int i = 0; i < SP_NQ; ++i) {
                g[i] = s->g[i * n + k];
                sum += g[i];
                mx += SP_CX[i] * g[i];
                my += SP_CY[i] * g[i];
            }
            double S = s->S[k], Fx = s->Fx[k], Fy = s->Fy[k];
            double rho, ux, uy;
            if (P->scheme == 0) {
                /* eq. (27aa) with rho~ = rho, and eq. (27a) with F = F_ext - lambda rho u, which
                 * is implicit in u; linear, so solved: rho u (1 + lambda/2) = sum c g + F_ext/2 */
                rho = sum + 0.5 * S;
                ux = (mx + 0.5 * Fx) / (rho * (1.0 + 0.5 * P->drag));
                uy = (my + 0.5 * Fy) / (rho * (1.0 + 0.5 * P->drag));
            } else {
                /* Remark 4 evolves f~ itself: rho~ = sum f~, rho u = sum c f~ (after eq. 21bb) */
                rho = sum;
                ux = mx / rho;
                uy = my / rho;
            }
            Fx -= P->drag * rho * ux;
            Fy -= P->drag * rho * uy;
            double Q = 2.0 / SP_DIM * rho * SP_CS2 - P->xi / (tau - 0.5);
            double divu = s->w1[k] + s->w2[k];
            double axx, axy, ayy, G[SP_NQ];
            /* p = rho c_s^2 = rho~ c_s^2: no d_t term; F~ = F; S~ = S */
            sp_bracket(0.0, ux, uy, Fx, Fy, P->full ? S : 0.0, Q, divu, &axx, &axy, &ayy);
            sp_force_distribution(S, Fx, Fy, axx, axy, ayy, G);
            for (int i = 0; i < SP_NQ; ++i) s->G[i * n + k] = G[i];
            s->rho[k] = rho;
            s->ux[k] = ux;
            s->uy[k] = uy;
            s->p[k] = rho * SP_CS2;
        }
    } else {
        /* grad p of the previous step (reading "full") */
        sp_gradient(P, s->p_prev, s->w1, s->w2);
        for (size_t k = 0; k < n; ++k) {
            double g[SP_NQ], mx = 0.0, my = 0.0;
            for (int i = 0; i < SP_NQ; ++i) {
                g[i] = s->g[i * n + k];
                mx += SP_CX[i] * g[i];
                my += SP_CY[i] * g[i];
            }
            double S = s->S[k], Fx = s->Fx[k], Fy = s->Fy[k];
            double ux = mx + 0.5 * Fx, uy = my + 0.5 * Fy; /* eq. (27a), rho = 1 */
            double Q = 2.0 / SP_DIM * SP_CS2 - P->xi / (tau - 0.5);
            double axx, axy, ayy, G[SP_NQ], p;
            if (P->full) {
                /* bracket without its d_t p I part, then eq. (28) with d_t p = p - p^{n-1}:
                 * the force term at i = 0 is G_0 = G_0' + w_0 (0 - c_s^2 I) : (d_t p I) / (2 c_s^4)
                 * = G_0' - w_0 d d_t p / (2 c_s^2); eq. (28), p = a [B + (tau - 1/2) G_0] with
                 * a = c_s^2 / (1 - w_0), is then p = X - c (p - p^{n-1}), solved for p */
                sp_bracket(0.0, ux, uy, Fx - s->w1[k], Fy - s->w2[k], S, Q, S, &axx, &axy, &ayy);
                sp_force_distribution(S, Fx, Fy, axx, axy, ayy, G);
                double X = sp_pressure_inc(g, S, ux, uy, tau, G[0], P->pscheme);
                double c = (P->pscheme == 0)
                               ? SP_CS2 / (1.0 - SP_W[0]) * (tau - 0.5) * SP_W[0] * SP_DIM / (2.0 * SP_CS2)
                               : 0.0;
                p = (X + c * s->p_prev[k]) / (1.0 + c);
                double dtp = p - s->p_prev[k];
                sp_bracket(dtp, ux, uy, Fx - s->w1[k], Fy - s->w2[k], S, Q, S, &axx, &axy, &ayy);
                sp_force_distribution(S, Fx, Fy, axx, axy, ayy, G);
            } else {
                sp_bracket(0.0, ux, uy, Fx, Fy, 0.0, Q, S, &axx, &axy, &ayy);
                sp_force_distribution(S, Fx, Fy, axx, axy, ayy, G);
                p = sp_pressure_inc(g, S, ux, uy, tau, G[0], P->pscheme);
            }
            for (int i = 0; i < SP_NQ; ++i) s->G[i * n + k] = G[i];
            s->rho[k] = 1.0;
            s->ux[k] = ux;
            s->uy[k] = uy;
            s->p[k] = p;
        }
    }
}

static void sp_one_step(sp_state* s) {
    const sp_params* P = &s->P;
    size_t n = s->n;
    int nx = P->nx, ny = P->ny;
    double tau = s->tau;
    sp_macroscopics(s);
    for (size_t k = 0; k < n; ++k) {
        double geq[SP_NQ];
        if (P->model == 0) sp_equilibrium_ni(s->rho[k], s->ux[k], s->uy[k], geq);
        else sp_equilibrium_inc(P->rho0, s->p[k], s->ux[k], s->uy[k], geq);
        for (int i = 0; i < SP_NQ; ++i) {
            double gi = s->g[i * n + k];
            if (P->scheme == 0) {
                /* eq. (24), dt = 1 */
                s->gs[i * n + k] = gi - (gi - geq[i]) / tau + (1.0 - 1.0 / (2.0 * tau)) * s->G[i * n + k];
            } else {
                /* Remark 4: f~* = f~ - (f~ - f^eq)/tau + G_i(x, t) + [G_i(x + c_i, t) - G_i(x, t - 1)] / 2;
                 * G_i(x + c_i) of a link that leaves the domain through a wall is taken at x;
                 * before the first step G(t - 1) = G(t) */
                int x = (int)(k % nx), j = (int)(k / nx);
                int xn = ((x + SP_CX[i]) % nx + nx) % nx, jn = j + SP_CY[i];
                size_t kn;
                if (P->bc == 0) kn = (size_t)(((jn % ny) + ny) % ny) * nx + xn;
                else kn = (jn < 0 || jn >= ny) ? k : (size_t)jn * nx + xn;
                double Gc = s->G[i * n + k], Gn = s->G[i * n + kn];
                double Gp = s->step == 0 ? Gc : s->G_prev[i * n + k];
                s->gs[i * n + k] = gi - (gi - geq[i]) / tau + Gc + 0.5 * (Gn - Gp);
            }
        }
    }
    for (int j = 0; j < ny; ++j)
        for (int x = 0; x < nx; ++x) {
            size_t k = (size_t)j * nx + x;
            for (int i = 0; i < SP_NQ; ++i) {
                int xd = ((x + SP_CX[i]) % nx + nx) % nx, jd = j + SP_CY[i];
                size_t dst;
                int idir = i;
                if (P->bc == 0) {
                    jd = ((jd % ny) + ny) % ny;
                    dst = (size_t)jd * nx + xd;
                } else if (jd < 0 || jd >= ny) {
                    idir = sp_opposite(i);
                    dst = k;
                } else {
                    dst = (size_t)jd * nx + xd;
                }
                s->g[idir * n + dst] = s->gs[i * n + k];
            }
        }
    for (size_t k = 0; k < n; ++k) {
        s->ux_prev[k] = s->ux[k];
        s->uy_prev[k] = s->uy[k];
        s->p_prev[k] = s->p[k];
    }
    memcpy(s->G_prev, s->G, SP_NQ * n * sizeof(double));
    s->step += 1;
}

void sp_step(sp_state* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) sp_one_step(s);
}

int64_t sp_step_count(const sp_state* s) { return s->step; }

/* Fields of the current state: 0 rho (model 0: rho~ = rho; model 1: 1), 1 u_x, 2 u_y, 3 p */
int sp_read(sp_state* s, int field, double* out) {
    sp_macroscopics(s);
    double* src[] = {s->rho, s->ux, s->uy, s->p};
    if (field < 0 || field > 3) return -1;
    memcpy(out, src[field], s->n * sizeof(double));
    return 0;
}

void sp_read_force_distribution(sp_state* s, double* out) {
    sp_macroscopics(s);
    memcpy(out, s->G, SP_NQ * s->n * sizeof(double));
}

/* sum over the grid of rho~: sum_i g_i + S/2 by eq. (27aa), sum_i f~_i under Remark 4 */
double sp_sum_rho_tilde(const sp_state* s) {
    double acc = 0.0;
    for (size_t k = 0; k < s->n; ++k) {
        for (int i = 0; i < SP_NQ; ++i) acc += s->g[i * s->n + k];
        if (s->P.scheme == 0) acc += 0.5 * s->S[k];  /* eq. (27aa); Remark 4: rho~ = sum f~ */
    }
    return acc;
}

void sp_get_state(const sp_state* s, double* g) { memcpy(g, s->g, SP_NQ * s->n * sizeof(double)); }
