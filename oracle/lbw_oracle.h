/*
 * lbw_oracle.h -- plain FP64 CPU oracle of the coupled lattice-Boltzmann +
 * finite-difference transport step (Lemus et al., "Modelling settling-driven
 * gravitational instabilities at the base of volcanic clouds using the
 * lattice Boltzmann method", arXiv 2106.07694).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP path; it exists to be checked against
 * the paper's closed forms and invariants and then to check the GPU path.
 *
 * Layout of every field (same convention as the product library, stated
 * independently here): x fastest, then y, then z; populations f[q][z][y][x].
 * The vertical axis (gravity, walls) is y in 2D and z in 3D.
 *
 * Every routine returns 0 on success and a negative value on bad arguments.
 *
 * Pins (tests/test_oracle_*.py): closed forms and invariants for every part.
 * The ghost values the WENO stencils see beyond a wall (mirrored scalar,
 * sign-flipped vertical fluid velocity, settling kept downward) are pinned by
 * a mirror image: a walled run's faces equal those of a periodic run of twice
 * the height holding the run and its reflection (eq. 14-15 as data).
 */
#ifndef LBW_ORACLE_H
#define LBW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_CLASSES 8

/* With n_classes >= 2 there are that many particle size classes (eq. 11-12):
 * each has its own concentration field, settling speed vs_class[i] and
 * diffusivity kappa_class[i] and obeys the C equation on its own; the force
 * uses the total concentration, -gp_c * sum_i C_i.  c then holds the class
 * fields one after the other (n_classes * N values) and the deposit one
 * counter per class and bottom column (n_classes * ncol).  n_classes 0 or 1:
 * a single class with vs and kappa_c. */
typedef struct {
    int32_t q;             /* 9 (D2Q9, 2D) or 19 (D3Q19, 3D) */
    int32_t nx, ny, nz;    /* nz == 1 in 2D */
    int32_t vert_periodic; /* 1: vertical axis periodic instead of walls */
    int32_t frozen;        /* 1: fluid step skipped, node velocity from u_in */
    int32_t scheme_c;      /* 0 WENO5-JS, 1 WENO3-JS, 2 first-order upwind */
    int32_t has_s;         /* second scalar S (upwind, forward Euler) */
    int32_t shifted;       /* populations stored as g_i = f_i - w_i */
    int32_t n_classes;     /* particle size classes, 0..ORC_MAX_CLASSES (0, 1: one) */
    double tau;            /* BGK relaxation time, > 1/2 */
    double body_force[3];  /* constant force density */
    double u_top[3];       /* top-wall velocity (moving lid) */
    double vs;             /* settling speed (downward) */
    double kappa_c, gp_c;  /* C diffusivity; vertical force -gp_c*C */
    double kappa_s, gp_s;  /* S diffusivity; vertical force -gp_s*S */
    double weno_eps;       /* WENO regularisation epsilon */
    double vs_class[ORC_MAX_CLASSES];    /* per-class settling speed (n_classes >= 2) */
    double kappa_class[ORC_MAX_CLASSES]; /* per-class diffusivity (n_classes >= 2) */
    /* The full force and settling of the paper (need has_s; 0 = off):
     * vs_s: the Stokes settling speed in fluid of density rho(S) (eq. 13,
     *   rho linear in S): every class settles at Vs (1 - vs_s S) with S at
     *   the node, so the conservative flux carries the -phi d(Vs)/dz term of
     *   eq. 7;
     * phi_c: particle volume fraction per unit C; the buoyancy of S acts on
     *   the fluid fraction, -gp_s S (1 - phi_c C) (eq. 10). */
    double vs_s;
    double phi_c;
} orc_cfg;

/* Lattice table in the documented order: c[q][3], w[q], opp[q]. */
int orc_lattice(int32_t q, int32_t *c, double *w, int32_t *opp);

/* f <- equilibrium at density rho (NULL: 1) and velocity u[dim][N] (NULL: 0). */
int orc_equilibrium(const orc_cfg *cfg, const double *rho, const double *u, double *f);

/* rho[N] and u[dim][N] (force-shifted velocity) from f, c, s. */
int orc_moments(const orc_cfg *cfg, const double *f, const double *c,
                const double *s, double *rho, double *u);

/* Spatial operator of the C equation for node velocity u[dim][N] and the
 * constant settling speed vs: out[N] = L(a); outflow[columns] = settling
 * flux through the bottom wall. */
int orc_rhs_c(const orc_cfg *cfg, const double *a, const double *u,
              double *out, double *outflow);

/* Face fluxes of the C equation (one size class): phi[ax][N] is the flux
 * through the +ax face of each node (advective WENO or upwind part minus the
 * central diffusion; the face of the top wall carries none) and bottom[ncol]
 * the flux through the bottom wall face that the operator differences, the
 * absorbed settling flux -Vs a_0 (0 with a periodic vertical axis, where the
 * bottom face of a column is the +face of its top node).  s is read only
 * when vs_s != 0 (settling speed Vs (1 - vs_s S)).  L(a) of orc_rhs_c is
 * minus the divergence of these faces. */
int orc_faces_c(const orc_cfg *cfg, const double *a, const double *u, const double *s,
                double *phi, double *bottom);

/* Advance nsteps coupled steps in place.  dep has one entry per size class
 * and bottom column (nx in 2D, nx*ny in 3D).  u_in is read in frozen mode; u_out
 * (optional) receives the node velocity used by the last step. */
int orc_run(const orc_cfg *cfg, double *f, double *c, double *s, double *dep,
            const double *u_in, double *u_out, int32_t nsteps);

/* Reverse-mode adjoint of one coupled step n -> n+1 (hand-written
 * transpose of steps 1-5; WENO5 only, no S).  Inputs: the forward state at n
 * (f_n, c_n) and the adjoints of the outputs (fbar_next of f^{n+1}, cbar_next
 * of C^{n+1}, dep_bar of every deposit counter).  Outputs: fbar, cbar (the
 * adjoints of f^n and C^n) and *vs_bar += dJ/dVs of this step.  In frozen
 * mode u_in is the node velocity and fbar/fbar_next are not used.  The upwind
 * side of every face is held at its forward choice. */
/* (One size class only.) */
int orc_adjoint_step(const orc_cfg *cfg, const double *f_n, const double *c_n,
                     const double *u_in, const double *fbar_next, const double *cbar_next,
                     double dep_bar, double *fbar, double *cbar, double *vs_bar);

/* out[0..3] = sum C, sum S, sum rho, sum dep (plain sequential sums; C and
 * dep over every size class). */
int orc_sums(const orc_cfg *cfg, const double *f, const double *c,
             const double *s, const double *dep, double *out);

/* Front of the particle field per bottom column (section "Comparison of
 * model results with predictions from linear stability analysis"): the
 * lowest height where C (the total over the size classes) reaches thr, measured from the bottom wall (cell v
 * has its centre at height v + 1/2), linear between the two cells that
 * straddle thr; 0 if the bottom cell already holds C >= thr, the domain
 * height if no cell does.  out[ncol]. */
int orc_front_height(const orc_cfg *cfg, const double *c, double thr, double *out);

/* Particle mass (sum of C, every size class) in the planes below plane
 * index `plane`, i.e. in
 * the cells with vertical index v < plane (the mass whose change gives the
 * flux through a horizontal plane, eq. for J in section "Particle mass flux,
 * particle concentration in the lower layer and accumulation rate"). */
int orc_mass_below(const orc_cfg *cfg, const double *c, int plane, double *out);

/* Power spectral density of a front height H[ncol] (as orc_front_height
 * writes it) along one lateral axis, the diagnostic the paper fits growth
 * rates to (eq. 45-46): for the slice of L samples along `axis` (0: x,
 * length nx; 1: y, length ny, 3D only) at index `index` of the other
 * lateral axis, Gamma(k) = |sum_j H_j exp(-2 pi i k j / L)|^2 / (kS L) for
 * k = 0 .. L/2 with kS = 1 (one sample per lattice spacing).  index = -1
 * averages Gamma over every slice along that axis.  out[L/2 + 1].  Returns
 * -1 for an invalid axis or index. */
int orc_front_psd(const orc_cfg *cfg, const double *h, int axis, int index, double *out);

#ifdef __cplusplus
}
#endif
#endif
