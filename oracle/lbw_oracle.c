/*
 * lbw_oracle.c -- plain FP64 CPU oracle of the coupled LBM + WENO step of
 * arXiv 2106.07694 (Lemus et al.).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written for
 * readability, not speed: two-lattice streaming, explicit ghost rules, face
 * fluxes stored per axis and then differenced, one loop per equation.
 *
 * What one step computes (section 2.3 of the paper and supplement section 1):
 *   1. moments of the populations (eq. 19-20) with the Guo half-force shift
 *      (eq. 22) -> rho, u; buoyancy force from C (and S) (eq. 10, linearised);
 *   2. C <- TVD-RK3 (S21-S23) of the conservative advection-diffusion-settling
 *      equation (eq. 6) with WENO face fluxes (S8-S20 gives the third-order
 *      form; the fifth-order Jiang-Shu form is the default here), velocity
 *      u - Vs e_vert frozen at time level n, absorbing bottom wall feeding the
 *      per-column deposit counter;
 *   3. S <- forward Euler of the first-order upwind conservative scheme
 *      (S5-S6 in conservative form) with central diffusion;
 *   4. BGK collision (eq. 18) with Guo forcing (eq. 22);
 *   5. streaming with half-way bounce-back at the walls (section 2.3.1), the
 *      moving-wall correction at the top.
 * All in lattice units: dx = dt = 1, cs^2 = 1/3 (eq. 21), rho0 = 1.
 *
 * Parity pins: every routine is exercised by the CPU tests against closed
 * forms or invariants.  The wall ghost rules of the WENO stencils are pinned
 * by a mirror image: every face of a walled run equals the same face of a
 * periodic run of twice the height that holds the run and its reflection
 * (the Neumann and no-penetration conditions of eq. 14-15 written out as
 * data), the wall faces aside.
 */
#include "lbw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 19

typedef struct {
    int q, dim, vert;
    int n[3];
    long N;       /* nodes */
    long ncol;    /* bottom columns */
    int ncls;     /* particle size classes (>= 1) */
    int c[MAXQ][3];
    double w[MAXQ];
    int opp[MAXQ];
} grid_t;

/* ----------------------------------------------------------------------- */
/* Lattices.  D2Q9: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-).      */
/* D3Q19: rest, +x, -x, +y, -y, +z, -z, then the 12 edge vectors in pairs  */
/* of opposites.  Weights are the standard second-order ones (the paper    */
/* cites Kruger et al. for the lattices; Fig. 3 shows D3Q19).              */
/* ----------------------------------------------------------------------- */
static int set_lattice(int q, grid_t *g)
{
    static const int c9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                 {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    static const int c19[19][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    int i, j;
    memset(g->c, 0, sizeof(g->c));
    if (q == 9) {
        g->q = 9;
        g->dim = 2;
        for (i = 0; i < 9; i++) {
            g->c[i][0] = c9[i][0];
            g->c[i][1] = c9[i][1];
            g->w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else if (q == 19) {
        g->q = 19;
        g->dim = 3;
        for (i = 0; i < 19; i++) {
            for (j = 0; j < 3; j++) g->c[i][j] = c19[i][j];
            g->w[i] = (i == 0) ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    } else {
        return -1;
    }
    /* opposite direction found by search, not tabulated */
    for (i = 0; i < g->q; i++) {
        g->opp[i] = -1;
        for (j = 0; j < g->q; j++)
            if (g->c[j][0] == -g->c[i][0] && g->c[j][1] == -g->c[i][1] &&
                g->c[j][2] == -g->c[i][2])
                g->opp[i] = j;
    }
    g->vert = g->dim - 1;
    return 0;
}

static int setup(const orc_cfg *cfg, grid_t *g)
{
    if (!cfg) return -1;
    if (set_lattice(cfg->q, g)) return -1;
    g->n[0] = cfg->nx;
    g->n[1] = cfg->ny;
    g->n[2] = cfg->nz;
    if (g->dim == 2 && cfg->nz != 1) return -1;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return -1;
    if (g->n[g->vert] < 6) return -1;
    if (cfg->n_classes < 0 || cfg->n_classes > ORC_MAX_CLASSES) return -1;
    if ((cfg->vs_s != 0.0 || cfg->phi_c != 0.0) && !cfg->has_s) return -1;
    g->ncls = cfg->n_classes > 1 ? cfg->n_classes : 1;
    g->N = (long)cfg->nx * cfg->ny * cfg->nz;
    g->ncol = (g->dim == 2) ? cfg->nx : (long)cfg->nx * cfg->ny;
    return 0;
}

static long node_index(const grid_t *g, const int p[3])
{
    return (long)p[0] + (long)g->n[0] * ((long)p[1] + (long)g->n[1] * p[2]);
}

static void node_coords(const grid_t *g, long k, int p[3])
{
    p[0] = (int)(k % g->n[0]);
    p[1] = (int)((k / g->n[0]) % g->n[1]);
    p[2] = (int)(k / ((long)g->n[0] * g->n[1]));
}

static long column_of(const grid_t *g, const int p[3])
{
    return (g->dim == 2) ? p[0] : (long)p[0] + (long)g->n[0] * p[1];
}

/* ----------------------------------------------------------------------- */
/* Moments, eq. 19-20 with the Guo shift rho u = sum f c + F/2 (eq. 22).    */
/* Force (eq. 10, linear in C and S): F = body + e_vert(-gp_c C -         */
/* gp_s S (1 - phi_c C)), C the total over the size classes (eq. 11-12).  */
/* ----------------------------------------------------------------------- */
static void force_at(const grid_t *g, const orc_cfg *cfg, const double *c,
                     const double *s, long k, double F[3])
{
    double ctot = 0.0;   /* total particle concentration, eq. 12 */
    int d, i;
    for (d = 0; d < 3; d++) F[d] = cfg->body_force[d];
    for (i = 0; i < g->ncls; i++) ctot += c[(long)i * g->N + k];
    F[g->vert] += -cfg->gp_c * ctot;
    /* the fluid's density anomaly acts on the fluid fraction 1 - phi,
       phi = phi_c * C (eq. 10) */
    if (cfg->has_s) F[g->vert] += -cfg->gp_s * (s[k] * (1.0 - cfg->phi_c * ctot));
}

static void moments_at(const grid_t *g, const orc_cfg *cfg, const double *f,
                       const double *c, const double *s, long k, double *rho,
                       double u[3], double F[3])
{
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    int i, d;
    for (i = 0; i < g->q; i++) {
        double fi = f[(long)i * g->N + k];
        r += fi;
        for (d = 0; d < 3; d++) m[d] += fi * g->c[i][d];
    }
    if (cfg->shifted) r = 1.0 + r; /* sum of w_i is 1 and sum w_i c_i is 0 */
    force_at(g, cfg, c, s, k, F);
    for (d = 0; d < 3; d++) u[d] = (m[d] + 0.5 * F[d]) / r;
    *rho = r;
}

/* ----------------------------------------------------------------------- */
/* Face reconstructions.  h are node fluxes ordered upwind -> downwind, a   */
/* the transported values in the same order (smoothness is measured on a). */
/* ----------------------------------------------------------------------- */

/* WENO5-JS (Jiang & Shu 1996): value at the right face of the centre node
 * of the five-node stencil; the fifth-order counterpart of S10-S16. */
static double weno5(const double h[5], const double a[5], double eps)
{
    double q0 = (2.0 * h[0] - 7.0 * h[1] + 11.0 * h[2]) / 6.0;
    double q1 = (-h[1] + 5.0 * h[2] + 2.0 * h[3]) / 6.0;
    double q2 = (2.0 * h[2] + 5.0 * h[3] - h[4]) / 6.0;
    double t, u;
    double b0, b1, b2, al0, al1, al2;
    t = a[0] - 2.0 * a[1] + a[2];
    u = a[0] - 4.0 * a[1] + 3.0 * a[2];
    b0 = 13.0 / 12.0 * t * t + 0.25 * u * u;
    t = a[1] - 2.0 * a[2] + a[3];
    u = a[1] - a[3];
    b1 = 13.0 / 12.0 * t * t + 0.25 * u * u;
    t = a[2] - 2.0 * a[3] + a[4];
    u = 3.0 * a[2] - 4.0 * a[3] + a[4];
    b2 = 13.0 / 12.0 * t * t + 0.25 * u * u;
    al0 = 0.1 / ((eps + b0) * (eps + b0));
    al1 = 0.6 / ((eps + b1) * (eps + b1));
    al2 = 0.3 / ((eps + b2) * (eps + b2));
    return (al0 * q0 + al1 * q1 + al2 * q2) / (al0 + al1 + al2);
}

/* WENO3 (S10-S16): upwind two-node candidate (S11) with weight 1/3, central
 * candidate (S10) with weight 2/3; stencil order upwind -> downwind. */
static double weno3(const double h[3], const double a[3], double eps)
{
    double qu = 0.5 * (3.0 * h[1] - h[0]);
    double qc = 0.5 * (h[1] + h[2]);
    double bu = (a[1] - a[0]) * (a[1] - a[0]);
    double bc = (a[2] - a[1]) * (a[2] - a[1]);
    double au = (1.0 / 3.0) / ((eps + bu) * (eps + bu));
    double ac = (2.0 / 3.0) / ((eps + bc) * (eps + bc));
    return (au * qu + ac * qc) / (au + ac);
}

/* Node index displaced by k along axis ax from p, with lateral periodicity
 * and, on the vertical axis with walls, even reflection about the walls
 * (Neumann, eq. 14-15).  *ghost is set when the reflection was applied. */
static long displaced(const grid_t *g, const orc_cfg *cfg, const int p[3],
                      int ax, int k, int *ghost)
{
    int r[3] = {p[0], p[1], p[2]};
    int n = g->n[ax];
    int j = p[ax] + k;
    *ghost = 0;
    if (ax != g->vert || cfg->vert_periodic) {
        j = ((j % n) + n) % n;
    } else if (j < 0) {
        j = -1 - j;
        *ghost = 1;
    } else if (j >= n) {
        j = 2 * n - 1 - j;
        *ghost = 1;
    }
    r[ax] = j;
    return node_index(g, r);
}

/* Settling speed at node k: vs, or with vs_s != 0 the Stokes speed in the
 * local fluid density (eq. 13 with rho linear in S), vs (1 - vs_s S_k).
 * s is NULL for a scalar that does not settle by S. */
static double settling_at(const orc_cfg *cfg, const double *s, double vs, long k)
{
    if (!s || cfg->vs_s == 0.0) return vs;
    return vs * (1.0 - cfg->vs_s * s[k]);
}

/* Transport velocity along ax at a node: u_ax - Vs on the vertical axis.
 * Beyond a wall the vertical fluid velocity is mirrored with a sign change
 * (no penetration), while settling keeps its direction (k is the mirrored
 * node, so a variable settling speed sees the mirrored S). */
static double transport_velocity(const grid_t *g, const orc_cfg *cfg, const double *u,
                                 const double *s, long k, int ax, int ghost, double vs)
{
    double ua = u[(long)ax * g->N + k];
    if (ax == g->vert) {
        if (ghost) ua = -ua;
        return ua - settling_at(cfg, s, vs, k);
    }
    return ua;
}

/* Face flux through the face between p and p + e_ax for scheme `scheme`,
 * diffusivity kappa, settling vs (0 for S; s: the S field that sets a
 * variable settling speed, or NULL). */
static double interior_face_flux(const grid_t *g, const orc_cfg *cfg,
                                 int scheme, double kappa, double vs,
                                 const double *a, const double *u, const double *s,
                                 const int p[3], int ax)
{
    double hv[6], av[6], wv[6];
    int m, gh;
    long k;
    double wf, hhat;
    /* stencil nodes p-2 .. p+3 along ax */
    for (m = 0; m < 6; m++) {
        k = displaced(g, cfg, p, ax, m - 2, &gh);
        av[m] = a[k];
        wv[m] = transport_velocity(g, cfg, u, s, k, ax, gh, vs);
        hv[m] = wv[m] * av[m];
    }
    /* upwind direction: sign of the face velocity, ties go left (R11) */
    wf = 0.5 * (wv[2] + wv[3]);
    if (scheme == 0) {
        double hh[5], aa[5];
        if (wf >= 0.0) {
            for (m = 0; m < 5; m++) { hh[m] = hv[m]; aa[m] = av[m]; }
        } else {
            for (m = 0; m < 5; m++) { hh[m] = hv[5 - m]; aa[m] = av[5 - m]; }
        }
        hhat = weno5(hh, aa, cfg->weno_eps);
    } else if (scheme == 1) {
        double hh[3], aa[3];
        if (wf >= 0.0) {
            for (m = 0; m < 3; m++) { hh[m] = hv[m + 1]; aa[m] = av[m + 1]; }
        } else {
            for (m = 0; m < 3; m++) { hh[m] = hv[4 - m]; aa[m] = av[4 - m]; }
        }
        hhat = weno3(hh, aa, cfg->weno_eps);
    } else {
        hhat = (wf >= 0.0) ? hv[2] : hv[3];
    }
    return hhat - kappa * (av[3] - av[2]);
}

/* phi[ax][k]: flux through the +ax face of node k; the face of the top
 * wall carries no flux. */
static void face_fluxes(const grid_t *g, const orc_cfg *cfg, int scheme,
                        double kappa, double vs, const double *a, const double *u,
                        const double *s, double *phi)
{
    long k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->N; k++) {
        int p[3], d;
        node_coords(g, k, p);
        for (d = 0; d < g->dim; d++) {
            if (d == g->vert && !cfg->vert_periodic && p[d] == g->n[d] - 1)
                phi[(long)d * g->N + k] = 0.0; /* top wall: no flux */
            else
                phi[(long)d * g->N + k] =
                    interior_face_flux(g, cfg, scheme, kappa, vs, a, u, s, p, d);
        }
    }
}

/* L(a) = -sum over axes of (Phi_{j+1/2} - Phi_{j-1/2}).
 * absorbing = 1: the bottom wall face carries the settling flux -vs*a_0
 * (outflow per column returned); otherwise walls carry no flux. */
static void spatial_operator(const grid_t *g, const orc_cfg *cfg, int scheme,
                             double kappa, double vs, int absorbing,
                             const double *a, const double *u, const double *s,
                             double *L, double *outflow)
{
    double *phi = (double *)malloc(sizeof(double) * (size_t)g->dim * g->N);
    long k;
    face_fluxes(g, cfg, scheme, kappa, vs, a, u, s, phi);
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->N; k++) {
        int p[3], d, gh;
        double acc = 0.0;
        node_coords(g, k, p);
        for (d = 0; d < g->dim; d++) {
            double right = phi[(long)d * g->N + k], left;
            if (d == g->vert && !cfg->vert_periodic && p[d] == 0) {
                left = absorbing ? -settling_at(cfg, s, vs, k) * a[k] : 0.0; /* bottom wall face */
            } else {
                long km = displaced(g, cfg, p, d, -1, &gh);
                left = phi[(long)d * g->N + km];
            }
            acc += right - left;
        }
        L[k] = -acc;
    }
    if (outflow) {
        for (k = 0; k < g->ncol; k++) outflow[k] = 0.0;
        if (absorbing && !cfg->vert_periodic) {
            for (k = 0; k < g->N; k++) {
                int p[3];
                node_coords(g, k, p);
                if (p[g->vert] == 0) outflow[column_of(g, p)] = settling_at(cfg, s, vs, k) * a[k];
            }
        }
    }
    free(phi);
}

/* ----------------------------------------------------------------------- */
/* Collision, eq. 18 + 22 (BGK with Guo forcing), and streaming with        */
/* half-way bounce-back; the moving-wall term is -6 w_i rho_w c_i.u_wall.   */
/* ----------------------------------------------------------------------- */
static void collide_stream(const grid_t *g, const orc_cfg *cfg, const double *f,
                           const double *rho, const double *u,
                           const double *F, double *fnew)
{
    long k;
    double omega = 1.0 / cfg->tau;
    double guo = 1.0 - 0.5 / cfg->tau;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->N; k++) {
        int p[3], i, d;
        double uk[3], Fk[3], usq = 0.0, drho = 0.0;
        node_coords(g, k, p);
        for (d = 0; d < 3; d++) {
            uk[d] = u[(long)d * g->N + k];
            Fk[d] = F[(long)d * g->N + k];
            if (d >= g->dim) { uk[d] = 0.0; Fk[d] = 0.0; }
            usq += uk[d] * uk[d];
        }
        /* shifted populations: the density anomaly is the sum of the stored
           g_i itself (the same sum as in moments_at, before 1 is added), not
           (1 + sum) - 1, which would keep it only to the rounding of 1 */
        if (cfg->shifted)
            for (i = 0; i < g->q; i++) drho += f[(long)i * g->N + k];
        for (i = 0; i < g->q; i++) {
            double cu = 0.0, cF = 0.0, uF = 0.0, feq, Fi, fs;
            int t[3], wall = 0;
            for (d = 0; d < 3; d++) {
                cu += g->c[i][d] * uk[d];
                cF += g->c[i][d] * Fk[d];
                uF += uk[d] * Fk[d];
            }
            if (cfg->shifted)
                feq = g->w[i] * (drho + rho[k] * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
            else
                feq = g->w[i] * rho[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            Fi = guo * g->w[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
            fs = f[(long)i * g->N + k];
            fs = fs - omega * (fs - feq) + Fi;
            /* destination */
            for (d = 0; d < 3; d++) t[d] = p[d] + g->c[i][d];
            for (d = 0; d < g->dim; d++) {
                if (d != g->vert || cfg->vert_periodic) {
                    t[d] = ((t[d] % g->n[d]) + g->n[d]) % g->n[d];
                } else if (t[d] < 0) {
                    wall = -1;
                } else if (t[d] >= g->n[d]) {
                    wall = 1;
                }
            }
            if (wall == 0) {
                fnew[(long)i * g->N + node_index(g, t)] = fs;
            } else {
                double cuw = 0.0;
                if (wall == 1)
                    for (d = 0; d < 3; d++) cuw += g->c[i][d] * cfg->u_top[d];
                fnew[(long)g->opp[i] * g->N + k] = fs - 6.0 * g->w[i] * cuw;
            }
        }
    }
}

/* ----------------------------------------------------------------------- */
/* Public entry points                                                      */
/* ----------------------------------------------------------------------- */
int orc_lattice(int32_t q, int32_t *c, double *w, int32_t *opp)
{
    grid_t g;
    int i, d;
    if (set_lattice(q, &g)) return -1;
    for (i = 0; i < g.q; i++) {
        for (d = 0; d < 3; d++) c[3 * i + d] = g.c[i][d];
        w[i] = g.w[i];
        opp[i] = g.opp[i];
    }
    return 0;
}

int orc_equilibrium(const orc_cfg *cfg, const double *rho, const double *u, double *f)
{
    grid_t g;
    long k;
    if (setup(cfg, &g)) return -1;
    for (k = 0; k < g.N; k++) {
        double r = rho ? rho[k] : 1.0, uk[3] = {0.0, 0.0, 0.0}, usq = 0.0;
        int i, d;
        for (d = 0; d < g.dim; d++) {
            uk[d] = u ? u[(long)d * g.N + k] : 0.0;
            usq += uk[d] * uk[d];
        }
        for (i = 0; i < g.q; i++) {
            double cu = 0.0, feq;
            for (d = 0; d < 3; d++) cu += g.c[i][d] * uk[d];
            feq = g.w[i] * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            f[(long)i * g.N + k] = cfg->shifted ? feq - g.w[i] : feq;
        }
    }
    return 0;
}

int orc_moments(const orc_cfg *cfg, const double *f, const double *c,
                const double *s, double *rho, double *u)
{
    grid_t g;
    long k;
    if (setup(cfg, &g)) return -1;
    for (k = 0; k < g.N; k++) {
        double r, uk[3], F[3];
        int d;
        moments_at(&g, cfg, f, c, s, k, &r, uk, F);
        if (rho) rho[k] = r;
        for (d = 0; d < g.dim; d++) u[(long)d * g.N + k] = uk[d];
    }
    return 0;
}

/* Settling speed and diffusivity of size class i. */
static double class_vs(const orc_cfg *cfg, int i)
{
    return cfg->n_classes > 1 ? cfg->vs_class[i] : cfg->vs;
}

static double class_kappa(const orc_cfg *cfg, int i)
{
    return cfg->n_classes > 1 ? cfg->kappa_class[i] : cfg->kappa_c;
}

int orc_rhs_c(const orc_cfg *cfg, const double *a, const double *u,
              double *out, double *outflow)
{
    grid_t g;
    if (setup(cfg, &g)) return -1;
    spatial_operator(&g, cfg, cfg->scheme_c, cfg->kappa_c, cfg->vs, 1, a, u, NULL,
                     out, outflow);
    return 0;
}

int orc_faces_c(const orc_cfg *cfg, const double *a, const double *u, const double *s,
                double *phi, double *bottom)
{
    grid_t g;
    long k;
    if (setup(cfg, &g)) return -1;
    if (g.ncls != 1) return -1;
    if (cfg->vs_s != 0.0 && !s) return -1;
    face_fluxes(&g, cfg, cfg->scheme_c, cfg->kappa_c, cfg->vs, a, u,
                cfg->vs_s != 0.0 ? s : NULL, phi);
    for (k = 0; k < g.ncol; k++) bottom[k] = 0.0;
    if (!cfg->vert_periodic) {
        for (k = 0; k < g.N; k++) {
            int p[3];
            node_coords(&g, k, p);
            /* the same value the operator differences at the bottom wall */
            if (p[g.vert] == 0)
                bottom[column_of(&g, p)] =
                    -settling_at(cfg, cfg->vs_s != 0.0 ? s : NULL, cfg->vs, k) * a[k];
        }
    }
    return 0;
}

int orc_run(const orc_cfg *cfg, double *f, double *c, double *s, double *dep,
            const double *u_in, double *u_out, int32_t nsteps)
{
    grid_t g;
    long k, N;
    int step, d, i;
    double *rho, *u, *F, *a1, *a2, *L, *cn, *out0, *out1, *out2, *fnew;
    const double *sn = cfg->has_s ? s : NULL;   /* S at level n sets Vs (eq. 13) */
    if (setup(cfg, &g)) return -1;
    if (cfg->tau <= 0.5 || nsteps < 0) return -1;
    if (cfg->frozen && !u_in) return -1;
    if (cfg->has_s && !s) return -1;
    N = g.N;
    rho = (double *)malloc(sizeof(double) * N);
    u = (double *)calloc((size_t)3 * N, sizeof(double));
    F = (double *)calloc((size_t)3 * N, sizeof(double));
    a1 = (double *)malloc(sizeof(double) * N);
    a2 = (double *)malloc(sizeof(double) * N);
    L = (double *)malloc(sizeof(double) * N);
    cn = (double *)malloc(sizeof(double) * N);
    out0 = (double *)malloc(sizeof(double) * g.ncol);
    out1 = (double *)malloc(sizeof(double) * g.ncol);
    out2 = (double *)malloc(sizeof(double) * g.ncol);
    fnew = cfg->frozen ? NULL : (double *)malloc(sizeof(double) * g.q * N);

    for (step = 0; step < nsteps; step++) {
        /* 1. moments and force at time level n (used by C, S and collision) */
        if (cfg->frozen) {
            for (k = 0; k < (long)g.dim * N; k++) u[k] = u_in[k];
        } else {
#pragma omp parallel for schedule(static)
            for (k = 0; k < N; k++) {
                double uk[3], Fk[3];
                int dd;
                moments_at(&g, cfg, f, c, s, k, &rho[k], uk, Fk);
                for (dd = 0; dd < 3; dd++) {
                    u[(long)dd * N + k] = uk[dd];
                    F[(long)dd * N + k] = Fk[dd];
                }
            }
        }
        /* 2. each size class C_i: TVD-RK3 (S21-S23) with its own settling
              speed and diffusivity, velocity (and a settling speed set by
              S) frozen at level n over the substeps; the force above
              already holds the classes at level n */
        for (i = 0; i < g.ncls; i++) {
            double *ci = c + (long)i * N;
            const double vs = class_vs(cfg, i), kappa = class_kappa(cfg, i);
            spatial_operator(&g, cfg, cfg->scheme_c, kappa, vs, 1, ci, u, sn, L, out0);
            for (k = 0; k < N; k++) a1[k] = ci[k] + L[k];
            spatial_operator(&g, cfg, cfg->scheme_c, kappa, vs, 1, a1, u, sn, L, out1);
            for (k = 0; k < N; k++) a2[k] = 0.75 * ci[k] + 0.25 * a1[k] + 0.25 * L[k];
            spatial_operator(&g, cfg, cfg->scheme_c, kappa, vs, 1, a2, u, sn, L, out2);
            for (k = 0; k < N; k++)
                cn[k] = ci[k] / 3.0 + 2.0 / 3.0 * a2[k] + 2.0 / 3.0 * L[k];
            if (dep)
                for (k = 0; k < g.ncol; k++)
                    dep[(long)i * g.ncol + k] += out0[k] / 6.0 + out1[k] / 6.0 + 2.0 / 3.0 * out2[k];
            for (k = 0; k < N; k++) ci[k] = cn[k];
        }
        /* 3. S: forward Euler, first-order upwind, no settling, closed walls */
        if (cfg->has_s) {
            spatial_operator(&g, cfg, 2, cfg->kappa_s, 0.0, 0, s, u, NULL, L, NULL);
            for (k = 0; k < N; k++) s[k] = s[k] + L[k];
        }
        /* 4-5. collide and stream */
        if (!cfg->frozen) {
            collide_stream(&g, cfg, f, rho, u, F, fnew);
            memcpy(f, fnew, sizeof(double) * g.q * N);
        }
    }
    if (u_out)
        for (d = 0; d < g.dim; d++)
            for (k = 0; k < N; k++) u_out[(long)d * N + k] = u[(long)d * N + k];

    free(rho); free(u); free(F); free(a1); free(a2); free(L); free(cn);
    free(out0); free(out1); free(out2); free(fnew);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* Adjoint (reverse mode) of one step.  Plain scatter loops, sequential.     */
/* ----------------------------------------------------------------------- */

/* Reverse of weno5(): given gbar = dJ/d(face value), accumulate dJ/dh and the
 * part of dJ/da that flows through the smoothness indicators. */
static void weno5_reverse(const double h[5], const double a[5], double eps, double gbar,
                          double hbar[5], double abar[5])
{
    const double d[3] = {0.1, 0.6, 0.3};
    double q[3], t[3], s[3], b[3], e[3], al[3], S = 0.0, g = 0.0;
    double qbar[3], bbar[3];
    int k;
    q[0] = (2.0 * h[0] - 7.0 * h[1] + 11.0 * h[2]) / 6.0;
    q[1] = (-h[1] + 5.0 * h[2] + 2.0 * h[3]) / 6.0;
    q[2] = (2.0 * h[2] + 5.0 * h[3] - h[4]) / 6.0;
    t[0] = a[0] - 2.0 * a[1] + a[2];
    s[0] = a[0] - 4.0 * a[1] + 3.0 * a[2];
    t[1] = a[1] - 2.0 * a[2] + a[3];
    s[1] = a[1] - a[3];
    t[2] = a[2] - 2.0 * a[3] + a[4];
    s[2] = 3.0 * a[2] - 4.0 * a[3] + a[4];
    for (k = 0; k < 3; k++) {
        b[k] = 13.0 / 12.0 * t[k] * t[k] + 0.25 * s[k] * s[k];
        e[k] = eps + b[k];
        al[k] = d[k] / (e[k] * e[k]);
        S += al[k];
    }
    for (k = 0; k < 3; k++) g += al[k] * q[k];
    g /= S;
    /* g = sum al q / sum al:  dg/dq_k = al_k/S,  dg/dal_k = (q_k - g)/S,
       dal_k/db_k = -2 al_k / e_k */
    for (k = 0; k < 3; k++) {
        qbar[k] = gbar * al[k] / S;
        bbar[k] = gbar * (q[k] - g) / S * (-2.0 * al[k] / e[k]);
    }
    hbar[0] += 2.0 / 6.0 * qbar[0];
    hbar[1] += -7.0 / 6.0 * qbar[0] - 1.0 / 6.0 * qbar[1];
    hbar[2] += 11.0 / 6.0 * qbar[0] + 5.0 / 6.0 * qbar[1] + 2.0 / 6.0 * qbar[2];
    hbar[3] += 2.0 / 6.0 * qbar[1] + 5.0 / 6.0 * qbar[2];
    hbar[4] += -1.0 / 6.0 * qbar[2];
    /* b = 13/12 t^2 + 1/4 s^2: db/dt = 13/6 t, db/ds = 1/2 s */
    {
        double tb = 13.0 / 6.0 * t[0] * bbar[0], sb = 0.5 * s[0] * bbar[0];
        abar[0] += tb + sb;
        abar[1] += -2.0 * tb - 4.0 * sb;
        abar[2] += tb + 3.0 * sb;
        tb = 13.0 / 6.0 * t[1] * bbar[1];
        sb = 0.5 * s[1] * bbar[1];
        abar[1] += tb + sb;
        abar[2] += -2.0 * tb;
        abar[3] += tb - sb;
        tb = 13.0 / 6.0 * t[2] * bbar[2];
        sb = 0.5 * s[2] * bbar[2];
        abar[2] += tb + 3.0 * sb;
        abar[3] += -2.0 * tb - 4.0 * sb;
        abar[4] += tb + sb;
    }
}

/* Reverse of L(a) (C equation, WENO5, absorbing bottom) for adjoint lam of
 * the output: abar += lam^T dL/da, ubar += lam^T dL/du, *vsbar += lam^T dL/dVs. */
static void spatial_operator_reverse(const grid_t *g, const orc_cfg *cfg, const double *a,
                                     const double *u, const double *lam, double *abar,
                                     double *ubar, double *vsbar)
{
    const double vs = cfg->vs, kappa = cfg->kappa_c;
    long k;
    for (k = 0; k < g->N; k++) {
        int p[3], d, m, gh;
        node_coords(g, k, p);
        for (d = 0; d < g->dim; d++) {
            long idx[6], kr;
            int ghost[6];
            double av[6], wv[6], hv[6], hbar[6], abar_l[6], phibar, wf;
            if (d == g->vert && !cfg->vert_periodic && p[d] == g->n[d] - 1) continue; /* top wall */
            /* L_k = -(Phi_{k+1/2} - Phi_{k-1/2}): Phi_{k+1/2} enters L_k with -1
               and L_{k+e} with +1 */
            kr = displaced(g, cfg, p, d, 1, &gh);
            phibar = lam[kr] - lam[k];
            for (m = 0; m < 6; m++) {
                idx[m] = displaced(g, cfg, p, d, m - 2, &ghost[m]);
                av[m] = a[idx[m]];
                wv[m] = transport_velocity(g, cfg, u, NULL, idx[m], d, ghost[m], vs);
                hv[m] = wv[m] * av[m];
                hbar[m] = 0.0;
                abar_l[m] = 0.0;
            }
            wf = 0.5 * (wv[2] + wv[3]);
            {
                double hh[5], aa[5], hb[5] = {0, 0, 0, 0, 0}, ab[5] = {0, 0, 0, 0, 0};
                int map[5];
                for (m = 0; m < 5; m++) map[m] = (wf >= 0.0) ? m : 5 - m;
                for (m = 0; m < 5; m++) { hh[m] = hv[map[m]]; aa[m] = av[map[m]]; }
                weno5_reverse(hh, aa, cfg->weno_eps, phibar, hb, ab);
                for (m = 0; m < 5; m++) { hbar[map[m]] += hb[m]; abar_l[map[m]] += ab[m]; }
            }
            /* diffusion part -kappa (a_{j+1} - a_j) */
            abar_l[3] += -kappa * phibar;
            abar_l[2] += kappa * phibar;
            for (m = 0; m < 6; m++) {
                double wbar = hbar[m] * av[m];
                abar[idx[m]] += abar_l[m] + hbar[m] * wv[m];
                if (d == g->vert) {
                    /* w = u - vs directly, or -u(mirror) - vs beyond a wall */
                    ubar[(long)d * g->N + idx[m]] += ghost[m] ? -wbar : wbar;
                    *vsbar += -wbar;
                } else {
                    ubar[(long)d * g->N + idx[m]] += wbar;
                }
            }
        }
        /* bottom wall face: L_0 gains -vs a_0 */
        if (!cfg->vert_periodic && p[g->vert] == 0) {
            abar[k] += -vs * lam[k];
            *vsbar += -a[k] * lam[k];
        }
    }
}

int orc_adjoint_step(const orc_cfg *cfg, const double *f_n, const double *c_n,
                     const double *u_in, const double *fbar_next, const double *cbar_next,
                     double dep_bar, double *fbar, double *cbar, double *vs_bar)
{
    grid_t g;
    long k, N;
    double *rho, *u, *F, *a1, *a2, *L, *ubar, *abar1, *abar2, *lam, vsb = 0.0;
    const double vs = cfg->vs;
    if (setup(cfg, &g)) return -1;
    if (cfg->scheme_c != 0 || cfg->has_s || cfg->shifted < 0 || g.ncls > 1) return -1;
    if (cfg->frozen ? !u_in : (!f_n || !fbar_next || !fbar)) return -1;
    N = g.N;
    rho = (double *)calloc(N, sizeof(double));
    u = (double *)calloc((size_t)3 * N, sizeof(double));
    F = (double *)calloc((size_t)3 * N, sizeof(double));
    a1 = (double *)calloc(N, sizeof(double));
    a2 = (double *)calloc(N, sizeof(double));
    L = (double *)calloc(N, sizeof(double));
    ubar = (double *)calloc((size_t)3 * N, sizeof(double));
    abar1 = (double *)calloc(N, sizeof(double));
    abar2 = (double *)calloc(N, sizeof(double));
    lam = (double *)calloc(N, sizeof(double));

    /* forward recomputation: moments (time level n) and the RK stages */
    for (k = 0; k < N; k++) {
        double uk[3], Fk[3];
        int d;
        if (cfg->frozen) {
            for (d = 0; d < g.dim; d++) u[(long)d * N + k] = u_in[(long)d * N + k];
        } else {
            moments_at(&g, cfg, f_n, c_n, NULL, k, &rho[k], uk, Fk);
            for (d = 0; d < 3; d++) { u[(long)d * N + k] = uk[d]; F[(long)d * N + k] = Fk[d]; }
        }
    }
    spatial_operator(&g, cfg, 0, cfg->kappa_c, vs, 1, c_n, u, NULL, L, NULL);
    for (k = 0; k < N; k++) a1[k] = c_n[k] + L[k];
    spatial_operator(&g, cfg, 0, cfg->kappa_c, vs, 1, a1, u, NULL, L, NULL);
    for (k = 0; k < N; k++) a2[k] = 0.75 * c_n[k] + 0.25 * a1[k] + 0.25 * L[k];

    /* reverse of C+ = C/3 + 2/3 a2 + 2/3 L(a2) and of the deposit update */
    for (k = 0; k < N; k++) {
        cbar[k] = cbar_next[k] / 3.0;
        abar2[k] = 2.0 / 3.0 * cbar_next[k];
        lam[k] = 2.0 / 3.0 * cbar_next[k];
    }
    spatial_operator_reverse(&g, cfg, a2, u, lam, abar2, ubar, &vsb);
    if (!cfg->vert_periodic) {
        for (k = 0; k < N; k++) {
            int p[3];
            node_coords(&g, k, p);
            if (p[g.vert] != 0) continue;
            /* D+ = D + vs (C/6 + a1/6 + 2 a2/3) at the bottom cells */
            cbar[k] += vs / 6.0 * dep_bar;
            abar1[k] += vs / 6.0 * dep_bar;
            abar2[k] += 2.0 * vs / 3.0 * dep_bar;
            vsb += dep_bar * (c_n[k] / 6.0 + a1[k] / 6.0 + 2.0 / 3.0 * a2[k]);
        }
    }
    /* reverse of a2 = 3/4 C + 1/4 a1 + 1/4 L(a1) */
    for (k = 0; k < N; k++) {
        cbar[k] += 0.75 * abar2[k];
        abar1[k] += 0.25 * abar2[k];
        lam[k] = 0.25 * abar2[k];
    }
    spatial_operator_reverse(&g, cfg, a1, u, lam, abar1, ubar, &vsb);
    /* reverse of a1 = C + L(C) */
    for (k = 0; k < N; k++) {
        cbar[k] += abar1[k];
        lam[k] = abar1[k];
    }
    spatial_operator_reverse(&g, cfg, c_n, u, lam, cbar, ubar, &vsb);

    /* reverse of streaming, collision and moments */
    if (!cfg->frozen) {
        double omega = 1.0 / cfg->tau, guo = 1.0 - 0.5 / cfg->tau;
        for (k = 0; k < N; k++) {
            int p[3], i, d, a;
            double fs_bar[MAXQ], uk[3], Fk[3], usq = 0.0, rb = 0.0, ub[3], Fb[3], mb[3];
            node_coords(&g, k, p);
            for (d = 0; d < 3; d++) {
                uk[d] = (d < g.dim) ? u[(long)d * N + k] : 0.0;
                Fk[d] = (d < g.dim) ? F[(long)d * N + k] : 0.0;
                ub[d] = (d < g.dim) ? ubar[(long)d * N + k] : 0.0;
                Fb[d] = 0.0;
                usq += uk[d] * uk[d];
            }
            /* streaming sent f*_i(x) to slot i of x + c_i, or to slot opp(i)
               of x when x + c_i lies beyond a wall: pull the adjoint back */
            for (i = 0; i < g.q; i++) {
                int t[3], wall = 0;
                for (d = 0; d < 3; d++) t[d] = p[d] + g.c[i][d];
                for (d = 0; d < g.dim; d++) {
                    if (d != g.vert || cfg->vert_periodic)
                        t[d] = ((t[d] % g.n[d]) + g.n[d]) % g.n[d];
                    else if (t[d] < 0 || t[d] >= g.n[d])
                        wall = 1;
                }
                fs_bar[i] = wall ? fbar_next[(long)g.opp[i] * N + k]
                                 : fbar_next[(long)i * N + node_index(&g, t)];
            }
            /* f* = f - omega (f - feq(rho, u)) + G(u, F) */
            for (i = 0; i < g.q; i++) {
                double cu = 0.0, cF = 0.0, poly, feqb = omega * fs_bar[i], Gb = fs_bar[i];
                for (d = 0; d < 3; d++) { cu += g.c[i][d] * uk[d]; cF += g.c[i][d] * Fk[d]; }
                poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
                fbar[(long)i * N + k] = (1.0 - omega) * fs_bar[i];
                rb += feqb * g.w[i] * (1.0 + poly);
                for (a = 0; a < 3; a++) {
                    ub[a] += feqb * g.w[i] * rho[k] * (3.0 * g.c[i][a] + 9.0 * cu * g.c[i][a] - 3.0 * uk[a]);
                    ub[a] += Gb * guo * g.w[i] * (-3.0 * Fk[a] + 9.0 * g.c[i][a] * cF);
                    Fb[a] += Gb * guo * g.w[i] * (3.0 * (g.c[i][a] - uk[a]) + 9.0 * cu * g.c[i][a]);
                }
            }
            /* u = (m + F/2)/rho with m = sum f c and rho = sum f (+1 shifted) */
            for (a = 0; a < 3; a++) {
                mb[a] = ub[a] / rho[k];
                Fb[a] += 0.5 * ub[a] / rho[k];
                rb += -ub[a] * uk[a] / rho[k];
            }
            for (i = 0; i < g.q; i++) {
                double s = rb;
                for (a = 0; a < 3; a++) s += mb[a] * g.c[i][a];
                fbar[(long)i * N + k] += s;
            }
            /* F_vert = body - gp_c C */
            cbar[k] += -cfg->gp_c * Fb[g.vert];
        }
    }
    *vs_bar += vsb;
    free(rho); free(u); free(F); free(a1); free(a2); free(L); free(ubar);
    free(abar1); free(abar2); free(lam);
    return 0;
}

/* Total particle concentration (eq. 12) at node k: the sum over the size
 * classes in class order. */
static double total_c(const grid_t *g, const double *c, long k)
{
    double t = 0.0;
    int i;
    for (i = 0; i < g->ncls; i++) t += c[(long)i * g->N + k];
    return t;
}

int orc_front_height(const orc_cfg *cfg, const double *c, double thr, double *out)
{
    grid_t g;
    long col, plane;
    int v, nv;
    if (setup(cfg, &g)) return -1;
    nv = g.n[g.dim - 1];
    plane = g.ncol;                          /* cells per horizontal plane */
    for (col = 0; col < g.ncol; col++) {
        double h = (double)nv;               /* no cell reaches thr */
        for (v = 0; v < nv; v++) {
            double cv = total_c(&g, c, col + (long)v * plane);
            if (cv >= thr) {
                if (v == 0) {
                    h = 0.0;
                } else {
                    double cb = total_c(&g, c, col + (long)(v - 1) * plane);
                    /* crossing between the centres of cells v-1 and v */
                    h = (double)(v - 1) + 0.5 + (thr - cb) / (cv - cb);
                }
                break;
            }
        }
        out[col] = h;
    }
    return 0;
}

int orc_mass_below(const orc_cfg *cfg, const double *c, int plane, double *out)
{
    grid_t g;
    long k, n;
    int nv, i;
    if (setup(cfg, &g)) return -1;
    nv = g.n[g.dim - 1];
    if (plane < 0 || plane > nv) return -1;
    n = (long)plane * g.ncol;
    *out = 0.0;
    for (i = 0; i < g.ncls; i++)             /* every size class */
        for (k = 0; k < n; k++) *out += c[(long)i * g.N + k];
    return 0;
}

int orc_front_psd(const orc_cfg *cfg, const double *h, int axis, int index, double *out)
{
    const double two_pi = 6.28318530717958647692528676655900577;
    grid_t g;
    long stride, step;
    int len, nslice, s, s0, s1, j, k;
    if (setup(cfg, &g)) return -1;
    if (axis < 0 || axis > g.dim - 2) return -1;        /* lateral axes only */
    if (axis == 0) {                                    /* along x, rows y */
        len = g.n[0];
        nslice = g.dim == 3 ? g.n[1] : 1;
        step = 1;
        stride = g.n[0];
    } else {                                            /* along y, rows x */
        len = g.n[1];
        nslice = g.n[0];
        step = g.n[0];
        stride = 1;
    }
    if (index < -1 || index >= nslice) return -1;
    s0 = index < 0 ? 0 : index;
    s1 = index < 0 ? nslice : index + 1;
    for (k = 0; k <= len / 2; k++) {
        double acc = 0.0;
        for (s = s0; s < s1; s++) {
            double re = 0.0, im = 0.0;
            for (j = 0; j < len; j++) {
                /* exp(-2 pi i k j / L), phase reduced modulo L exactly */
                double ang = two_pi * (double)(((long)k * j) % len) / (double)len;
                double hj = h[(long)s * stride + (long)j * step];
                re += hj * cos(ang);
                im -= hj * sin(ang);
            }
            acc += (re * re + im * im) / (double)len;
        }
        out[k] = acc / (double)(s1 - s0);
    }
    return 0;
}

int orc_sums(const orc_cfg *cfg, const double *f, const double *c,
             const double *s, const double *dep, double *out)
{
    grid_t g;
    long k;
    int i;
    if (setup(cfg, &g)) return -1;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (k = 0; k < (long)g.ncls * g.N; k++) out[0] += c[k];   /* every size class */
    if (s)
        for (k = 0; k < g.N; k++) out[1] += s[k];
    if (f)
        for (k = 0; k < g.N; k++) {
            double r = cfg->shifted ? 1.0 : 0.0;
            for (i = 0; i < g.q; i++) r += f[(long)i * g.N + k];
            out[2] += r;
        }
    if (dep)
        for (k = 0; k < (long)g.ncls * g.ncol; k++) out[3] += dep[k];
    return 0;
}
