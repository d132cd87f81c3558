/*
 * lbw.h -- C ABI of liblbw.so: the coupled lattice-Boltzmann + WENO step of
 * Lemus et al., "Modelling settling-driven gravitational instabilities at the
 * base of volcanic clouds using the lattice Boltzmann method" (arXiv
 * 2106.07694), as hand-written HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * One time step (section 2.3 "Numerical methods" and supplement section 1):
 *   1. moments rho = sum f_i, rho u = sum f_i c_i + F/2 (eq. 19-20, Guo shift
 *      of eq. 22) and the buoyancy force F = body + e_v(-gp_c C - gp_s S)
 *      (eq. 10 linearised in C and S);
 *   2. particle concentration C: TVD-RK3 (S21-S23) of the conservative
 *      advection-diffusion-settling equation (eq. 6) with WENO face fluxes
 *      (S8-S20; fifth-order Jiang-Shu by default), transport velocity
 *      u - Vs e_v frozen at time level n, central diffusion, absorbing bottom
 *      wall whose settling flux accumulates in a per-column deposit counter;
 *   3. optional second scalar S (sugar): first-order upwind in conservative
 *      form (S5-S6), central diffusion, forward Euler, closed walls;
 *   4. BGK collision with Guo forcing (eq. 18, 22), tau = nu/cs^2 + 1/2
 *      (eq. 21), cs^2 = 1/3;
 *   5. streaming with half-way bounce-back at the bottom and top walls
 *      (section 2.3.1); a moving top wall adds -6 w_i c_i.u_top.
 * Lattice units throughout: dx = dt = 1, rho0 = 1.
 *
 * Geometry and layout.  Fields are structure-of-arrays with x fastest:
 * node index k = x + nx*(y + ny*z), N = nx*ny*nz.  Populations f[q][k]
 * (q-major), velocity u[d][k], scalars C[k], S[k].  The vertical axis (gravity,
 * walls) is y in 2D (nz = 1) and z in 3D; the lateral axes are periodic.
 * Deposit: one FP64 value per bottom column, index x (2D) or x + nx*y (3D).
 *
 * Population order (fixed):
 *   D2Q9:  0 rest; 1 (+1,0) 2 (0,+1) 3 (-1,0) 4 (0,-1)
 *          5 (+1,+1) 6 (-1,+1) 7 (-1,-1) 8 (+1,-1)
 *   D3Q19: 0 rest; 1 +x 2 -x 3 +y 4 -y 5 +z 6 -z
 *          7 (+1,+1,0) 8 (-1,-1,0) 9 (+1,-1,0) 10 (-1,+1,0)
 *          11 (+1,0,+1) 12 (-1,0,-1) 13 (+1,0,-1) 14 (-1,0,+1)
 *          15 (0,+1,+1) 16 (0,-1,-1) 17 (0,+1,-1) 18 (0,-1,+1)
 *
 * Precision.  LBW_FP64 stores f and computes in double.  LBW_FP32_SHIFTED
 * stores g_i = f_i - w_i (rho0 = 1) and computes in float; the deposit
 * counter and every reduction stay FP64.  LBW_FP64_SHIFTED is the shifted
 * algebra in double.
 *
 * Streaming is in place (two alternating kernels, "AA" access pattern): after
 * an odd number of steps the population buffer holds post-collision values in
 * swapped slots.  Read or write populations only through lbw_export /
 * lbw_import, which present the canonical pre-collision layout f_i(x, t).
 *
 * Ownership.  Every device buffer belongs to the caller and must outlive the
 * handle.  The library allocates no device memory (its one device array, the
 * fixed scratch of lbw_reduce_static, is part of its code object) and never
 * synchronises the stream except in the reductions.  Calls on one handle
 * must not overlap.
 *
 * Errors.  Every int-returning function returns LBW_OK (0) or a negative
 * LBW_ERR_* code; lbw_last_error() then describes the failure (thread-local
 * string, valid until the next call on the same thread).  No exception or
 * abort crosses the ABI.
 */
#ifndef LBW_H
#define LBW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBW_ABI_VERSION 3
#define LBW_MAX_CLASSES 8   /* particle size classes per run */

enum {
    LBW_OK = 0,
    LBW_ERR_INVAL = -1,       /* bad argument or configuration */
    LBW_ERR_UNSUPPORTED = -2, /* valid request the library does not provide */
    LBW_ERR_HIP = -3,         /* a HIP runtime call failed */
    LBW_ERR_NONFINITE = -4    /* a reduction found NaN or Inf */
};

enum { LBW_D2Q9 = 9, LBW_D3Q19 = 19 };
enum { LBW_FP64 = 0, LBW_FP32_SHIFTED = 1, LBW_FP64_SHIFTED = 2 };
enum { LBW_FLUID_LBM = 0, LBW_FLUID_FROZEN = 1 };
enum { LBW_WENO5 = 0, LBW_WENO3 = 1, LBW_UPWIND1 = 2 };
enum { LBW_FIELD_F = 0, LBW_FIELD_C = 1, LBW_FIELD_S = 2, LBW_FIELD_U = 3,
       LBW_FIELD_DEPOSIT = 4, LBW_FIELD_STAGE1 = 5, LBW_FIELD_STAGE2 = 6,
       LBW_FIELD_RHO = 7 };
enum { LBW_MASS_C = 0, LBW_MASS_S = 1, LBW_MASS_FLUID = 2, LBW_DEPOSIT = 3 };
enum { LBW_PHASE_COLLIDE_STREAM = 0, LBW_PHASE_TRANSPORT = 1, LBW_NPHASES = 2 };

/* One run's physics and grid (lattice units). */
typedef struct {
    int32_t lattice;       /* LBW_D2Q9 (2D, nz = 1) | LBW_D3Q19 (3D) */
    int32_t precision;     /* LBW_FP64 | LBW_FP32_SHIFTED | LBW_FP64_SHIFTED */
    int32_t nx, ny, nz;    /* nx, ny >= 1; vertical extent >= 6 */
    int32_t vert_periodic; /* 0: bounce-back walls bottom/top; 1: periodic */
    int32_t fluid_mode;    /* LBW_FLUID_LBM | LBW_FLUID_FROZEN (u is an input,
                              the populations are not touched) */
    int32_t scheme_c;      /* LBW_WENO5 | LBW_WENO3 | LBW_UPWIND1 for C */
    int32_t has_s;         /* 1: transport S and add its buoyancy */
    int32_t n_classes;     /* particle size classes (eq. 11-12): 0 or 1 for one
                              class with vs and kappa_c; 2..LBW_MAX_CLASSES:
                              class i settles at vs_class[i] and diffuses with
                              kappa_class[i] (vs and kappa_c must then be 0),
                              each obeys the C equation on its own, and the
                              buoyancy is that of the total, -gp_c sum_i C_i */
    double tau;            /* BGK relaxation time, > 1/2 (eq. 21) */
    double body_force[3];  /* constant force density */
    double u_top[3];       /* top-wall velocity (moving lid) */
    double vs;             /* settling speed >= 0 (downward) */
    double kappa_c, gp_c;  /* C diffusivity; vertical force -gp_c*C */
    double kappa_s, gp_s;  /* S diffusivity; vertical force -gp_s*S */
    double weno_eps;       /* WENO regularisation, > 0 (1e-6 typical) */
    double vs_class[LBW_MAX_CLASSES];    /* n_classes >= 2: settling speeds */
    double kappa_class[LBW_MAX_CLASSES]; /* n_classes >= 2: diffusivities */
    /* The paper's full force and settling (both need has_s; 0 = off):
     * vs_s   every class settles at its speed times (1 - vs_s S), S at the
     *        node: the Stokes speed in fluid of density rho(S) (eq. 13, rho
     *        linear in S).  The conservative face fluxes then carry the
     *        -phi d(Vs)/dz term of eq. 7.  The caller keeps |Vs| <= 1 over
     *        the S values the run reaches (S stays within its initial range);
     * phi_c  particle volume fraction per unit C: the buoyancy of S acts on
     *        the fluid fraction, -gp_s S (1 - phi_c C) (eq. 10). */
    double vs_s;
    double phi_c;
} lbw_config;

/* One run's device buffers (caller-owned, element type per precision:
 * double for the FP64 forms, float for LBW_FP32_SHIFTED; deposit is always
 * double).  Unused pointers may be NULL. */
typedef struct {
    void *f;           /* Q*N populations (in place, AA order) */
    void *c;           /* N per size class, class after class: C_i */
    void *c_s1;        /* N per size class: RK stage work buffer */
    void *c_s2;        /* N per size class: RK stage work buffer */
    void *s;           /* N: S (has_s) */
    void *s_tmp;       /* N: S work buffer (has_s) */
    void *u;           /* dim*N: node velocity of the last step; input when
                          fluid_mode = LBW_FLUID_FROZEN */
    double *deposit;   /* ncol per size class, class after class: settled
                          mass per bottom column (FP64) */
    void *scratch;     /* reduction partials, >= lbw_scratch_bytes() bytes */
    size_t scratch_bytes;
} lbw_buffers;

/* Launch shape of the hot kernels (chosen by the autotuner; 0 = default). */
typedef struct {
    int32_t lbm_block;     /* threads per block of the collide-stream kernel */
    int32_t tile_x;        /* transport tile width: 32, 64, 128 (3D) or
                              64, 128, 256, 512 (2D) columns */
    int32_t tile_y;        /* transport chunk: vertical planes per block */
    int32_t variant;       /* 0 tiled transport (LDS, marching) after the
                              collide-stream kernel; 1 plain transport (one
                              thread per node, no LDS) */
    int32_t graph;         /* 1: lbw_step replays a captured HIP graph of two
                              steps (needs a non-null stream; the graph is
                              runtime-owned and rebuilt after lbw_set_launch) */
    int32_t reserved;      /* must be 0 */
    int32_t tile_rows;     /* transport tile rows (3D): 0 = 256 / tile_x
                              (32x8, 64x4, 128x2 with 256 threads), or 16 with
                              tile_x 32 and 8 with tile_x 64 (512 threads);
                              2D tiles are one row (0 or 1) */
} lbw_launch;

/* Library ABI version (LBW_ABI_VERSION). */
int lbw_version(void);

/* Description of the last error on this thread ("" if none). */
const char *lbw_last_error(void);

/* Bytes of device scratch the runs need: reduction partials, plus, when
 * nbatch > 1, the device copy of the run table and the work lists of the
 * batched (persistent) kernels.  Batched runs must pass this scratch in
 * run 0's buffers at creation. */
int lbw_scratch_bytes(const lbw_config *cfgs, int32_t nbatch, size_t *out_bytes);

typedef struct lbw_handle lbw_handle;

/* Validate nbatch configurations and their buffers and bind them to a HIP
 * stream (a hipStream_t passed as void*; NULL = the null stream).
 * Rejects tau <= 1/2 (BGK stability, eq. 21 and the remark after eq. 23),
 * a vertical extent < 6 (one WENO5 stencil), negative vs or diffusivities,
 * kappa above the explicit-diffusion limit 1/(2 dim), |u_top| or vs above the
 * CFL bound (S7), weno_eps <= 0, NULL required buffers, and, when nbatch > 1,
 * runs of different lattice, precision, fluid mode, scheme or S option.
 * A run may hold up to 2^32 - 1024 cells (the per-cell kernels launch one
 * work-item per cell), with fewer than 2^29 cells in a horizontal plane
 * (lanes address a plane with 32-bit byte offsets).
 * Host memory only (freed by lbw_destroy).  *out is NULL on failure. */
int lbw_create(const lbw_config *cfgs, const lbw_buffers *bufs, int32_t nbatch,
               void *stream, lbw_handle **out);

/* Release the handle (host memory only).  NULL is accepted. */
void lbw_destroy(lbw_handle *h);

/* Choose the kernels' launch shape (the autotuner's knob).  Zero fields keep
 * the defaults; invalid shapes are rejected with LBW_ERR_INVAL, and so is a
 * shape whose tiled transport launch for a single run would need 2^32
 * work-items or more (one block per tile and vertical chunk). */
int lbw_set_launch(lbw_handle *h, const lbw_launch *launch);
int lbw_get_launch(const lbw_handle *h, lbw_launch *launch);

/* Populations of run `run` <- equilibrium at density rho[N] and velocity
 * u[dim][N] (device arrays of the run's element type; NULL means rho = 1,
 * u = 0), the initial state of section 2.2 (fluid at rest).  Written in the
 * layout the current in-place streaming parity expects (as lbw_import does),
 * so it may be called after any number of steps.  Asynchronous on the
 * handle's stream. */
int lbw_init_equilibrium(lbw_handle *h, int32_t run, const void *rho, const void *u);

/* Advance every run by nsteps coupled steps (nsteps >= 0; 0 does nothing).
 * Asynchronous on the handle's stream; no host synchronisation, no
 * allocation.  If a launch fails (LBW_ERR_HIP) the runs' state is undefined:
 * import or re-initialise it before stepping again. */
int lbw_step(lbw_handle *h, int32_t nsteps);

/* Number of steps taken since creation (imports do not change it). */
int lbw_steps_done(const lbw_handle *h, int64_t *out);

/* Copy field `field` of run `run` in canonical layout into the device buffer
 * dst (populations: pre-collision f_i(x, t) -- or g_i for the shifted forms --
 * in f[q][k] order; C: every size class, class after class; u: the last
 * step's node velocity; STAGE1, STAGE2: the last step's first and second RK
 * stages of C, every class; deposit: FP64 ncol per class).
 * Asynchronous on the handle's stream. */
int lbw_export(lbw_handle *h, int32_t run, int32_t field, void *dst);

/* Overwrite field `field` of run `run` from the canonical device buffer src
 * (same layouts as lbw_export).  Populations are written in the layout the
 * current in-place streaming parity expects; the parity and the step counter
 * are unchanged.  A state exported after an even number of
 * steps and imported into a fresh handle continues bit for bit as the
 * uninterrupted run; after an odd number the two continue with different
 * kernels of the in-place pair and agree to rounding.  Asynchronous on the
 * handle's stream. */
int lbw_import(lbw_handle *h, int32_t run, int32_t field, const void *src);

/* Point the buffer the step writes field `field` of run `run` into at the
 * caller's device array ptr (same size and layout as the one given at
 * creation; ptr NULL restores that one).  Only per-step outputs can be
 * rebound: LBW_FIELD_U (the node velocity of eq. 20, LBW_FLUID_LBM only,
 * since a frozen velocity is an input), LBW_FIELD_STAGE1 and
 * LBW_FIELD_STAGE2 (the first two TVD-RK3 stages, S21-S22), and
 * LBW_FIELD_RHO (the node density of eq. 19, LBW_FLUID_LBM only; N values of
 * the run's element type): the density has no buffer of its own and is
 * written only while bound (ptr NULL stops it).  From the next step on the
 * step writes them there, so a caller that keeps every step's
 * intermediates (the replay of a checkpointed adjoint) copies nothing.
 * Nothing is copied; ptr must stay valid while bound.  Drops a captured
 * graph; for a batch it re-uploads the work lists (synchronises the
 * stream).  Returns LBW_ERR_INVAL for any other field. */
int lbw_rebind(lbw_handle *h, int32_t run, int32_t field, void *ptr);

/* Replay n steps of run `run` from its current state, keeping what the
 * reverse steps of the adjoint read (S21-S23 and eq. 19-20 at each step):
 * before step i, C is copied into c_out[i] (every size class, as lbw_export
 * gives it); during step i the velocity, the density and the first two RK
 * stages are written into u_out[i], rho_out[i], a1_out[i] and a2_out[i].
 * The six arrays hold n device pointers each (host arrays of pointers, read
 * during the call); u_out and rho_out are NULL for LBW_FLUID_FROZEN.  It is n
 * rounds of lbw_export(C), lbw_rebind(U, RHO, STAGE1, STAGE2) and
 * lbw_step(1) without a host call per step; afterwards the four fields are
 * bound back to the buffers given at creation.  Asynchronous on the handle's
 * stream; the buffers must stay valid until that work has run.  Returns
 * LBW_ERR_INVAL for n < 0 or a NULL array or element where one is needed,
 * LBW_ERR_UNSUPPORTED for a batch (a step advances every run of it). */
int lbw_replay(lbw_handle *h, int32_t run, int32_t n, void *const *c_out, void *const *u_out,
               void *const *rho_out, void *const *a1_out, void *const *a2_out);

/* FP64 sums per run into out_host[nbatch]: LBW_MASS_C (sum C over every
 * size class), LBW_MASS_S (sum S), LBW_MASS_FLUID (sum rho), LBW_DEPOSIT
 * (sum of the deposit counters of every class), the particle mass and
 * deposited mass m_b of section 4.2.3.
 * Wavefront shuffles, per-block partials, then a fixed-order final pass:
 * the result is bitwise reproducible.  Synchronises the stream.  Returns
 * LBW_ERR_NONFINITE if any sum is NaN or Inf (the values are still written). */
int lbw_reduce(lbw_handle *h, int32_t what, double *out_host);

/* lbw_reduce for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid allocation, code that runs between graph replays):
 * the same sums, bit for bit, with the partial sums kept in a device array the
 * library holds itself instead of the scratch passed at creation, which may
 * then be NULL.  That array is static: 128 * 256 + 128 doubles (263,168
 * bytes) on every device the library runs on, held until the process ends,
 * enough for batches of up to 128 runs (LBW_ERR_INVAL beyond).  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * All calls on one device share that device's array and leave their partial
 * sums in it; each call writes every value it reads, so no clearing is
 * needed, but calls that overlap on one device (other threads, other
 * handles) race and must be serialised by the caller.  Synchronises the
 * stream (so it cannot itself be recorded into a graph); LBW_ERR_NONFINITE
 * as lbw_reduce. */
int lbw_reduce_static(lbw_handle *h, int32_t what, double *out_host);

/* The sums of lbw_reduce for one particle size class, per run, into
 * out_host[nbatch]: LBW_MASS_C (sum of C_cls) or LBW_DEPOSIT (the class's
 * deposit counters), i.e. the suspended and deposited mass of that class
 * (eq. 11-12; with one class, cls = 0 gives the lbw_reduce values).  Same
 * deterministic reduction; synchronises the stream.  LBW_ERR_INVAL for
 * another `what` or a class some run of the batch does not have;
 * LBW_ERR_NONFINITE as lbw_reduce. */
int lbw_reduce_class(lbw_handle *h, int32_t what, int32_t cls, double *out_host);

/* Particle mass below a horizontal plane, per run, into out_host[nbatch]:
 * the FP64 sum of C (every size class) over the cells whose vertical index
 * v is below `plane`
 * (the first plane * ncol nodes, planes being the slowest axis).  Its change
 * over an interval divided by the plane's area and the interval gives the
 * particle mass flux J through that plane (section "Particle mass flux,
 * particle concentration in the lower layer and accumulation rate"); plane
 * = nv gives the LBW_MASS_C total.  Same deterministic reduction as
 * lbw_reduce; synchronises the stream.  LBW_ERR_INVAL if plane is outside
 * [0, nv] for any run of the batch (nv = ny in 2D, nz in 3D);
 * LBW_ERR_NONFINITE as lbw_reduce. */
int lbw_mass_below(lbw_handle *h, int32_t plane, double *out_host);

/* Height of the particle front in every bottom column of run `run`, into the
 * caller's device array out_dev[ncol] (FP64; ncol = nx in 2D, nx*ny in 3D,
 * column index x + nx*y): scanning each column upward from the bottom wall,
 * the height where C (the total over the size classes, summed in FP64 in
 * class order) first reaches `threshold`, measured from the wall with
 * the centre of cell v at v + 1/2 and linear between the two cells that
 * straddle the threshold; 0 if the bottom cell already reaches it and the
 * domain height nv if no cell does.  Its lateral Fourier modes give the
 * finger growth of section "Comparison of model results with predictions
 * from linear stability analysis".  C is read in the run's storage type
 * and compared in FP64.  Enqueued on the handle's stream, no
 * synchronisation.  LBW_ERR_INVAL for a bad run, NULL out_dev or a
 * non-finite threshold. */
int lbw_front_height(lbw_handle *h, int32_t run, double threshold, double *out_dev);

/* Power spectral density of a front height along one lateral axis, the
 * spectrum the paper extracts dominant wavenumbers and growth rates from
 * (eq. 45-46 and the passage defining it): for the row of L samples of
 * height_dev (device, FP64, ncol values in the layout lbw_front_height
 * writes) along `axis` (0: x, L = nx; 1: y, L = ny, 3D runs only) at index
 * `index` of the other lateral axis,
 *   Gamma(k) = |sum_j H_j exp(-2 pi i k j / L)|^2 / (kS L),  k = 0 .. L/2,
 * with kS = 1 (one sample per lattice spacing), into the caller's device
 * array out_dev[L/2 + 1] (FP64).  index = -1 averages Gamma over every row
 * along that axis.  The sums run in a fixed order: the same input gives the
 * same bits.  Enqueued on the handle's stream.  LBW_ERR_INVAL for a bad run,
 * NULL pointers, an axis that is not lateral or an index outside [-1, rows). */
int lbw_front_psd(lbw_handle *h, int32_t run, const double *height_dev, int32_t axis,
                  int32_t index, double *out_dev);

/* Device workspace lbw_adjoint_step needs for run `run` (bytes). */
int lbw_adjoint_work_bytes(const lbw_handle *h, int32_t run, size_t *out_bytes);

/* Reverse mode of one coupled step n -> n+1 of run `run`: the hand-written
 * transpose of moments, RK3 transport (S21-S23, WENO5 weights differentiated
 * through their smoothness indicators, the upwind side of each face held at
 * its forward choice), deposit update, BGK + Guo collision and bounce-back
 * streaming.  For J a function of the state at n+1:
 *   f_n, c_n     forward state at n (canonical populations, as lbw_export
 *                writes them; C), device arrays of the run's element type;
 *                f_n may be NULL when u_n and rho_n are given;
 *   u_n, rho_n, a1_n, a2_n  optional forward intermediates of step n (its
 *                node velocity and density and first two RK stages, as the
 *                step writes them into buffers bound with lbw_rebind, or as
 *                lbw_export gives U, STAGE1, STAGE2 right after that step);
 *                NULL: recomputed from f_n and c_n (rho_n is used only
 *                together with u_n);
 *   fbar_next    dJ/df^{n+1} (canonical layout); cbar_next = dJ/dC^{n+1};
 *   dep_bar      dJ/d(deposit) of every column (1 for the total deposited
 *                mass m_b of section 4.2.3);
 *   fbar, cbar   out: dJ/df^n and dJ/dC^n (must not alias the inputs);
 *   work         device workspace of lbw_adjoint_work_bytes bytes, zero-filled
 *                by the caller before the first step of a sweep; it carries an
 *                FP64 per-node accumulator of dJ/dVs across steps;
 *   vs_bar_dev   NULL, or a device FP64 scalar: the accumulator is then
 *                summed in a fixed order, added to *vs_bar_dev and cleared.
 * WENO5 without S and with one size class only (LBW_ERR_UNSUPPORTED
 * otherwise).  In frozen mode the
 * run's u buffer is the (constant) velocity and the population arguments may
 * be NULL.  Asynchronous on the handle's stream; independent of the handle's
 * own state buffers apart from that velocity. */
int lbw_adjoint_step(lbw_handle *h, int32_t run, const void *f_n, const void *c_n,
                     const void *u_n, const void *rho_n, const void *a1_n, const void *a2_n,
                     const void *fbar_next, const void *cbar_next, double dep_bar, void *fbar,
                     void *cbar, double *vs_bar_dev, void *work, size_t work_bytes);

/* Per-phase GPU time of the lbw_step calls made between lbw_timing_begin and
 * lbw_timing_end: HIP events are recorded on the stream each launch goes to,
 * around every collide-stream launch and around the transport launches of
 * every step.  lbw_timing_end waits for the events and writes
 * the summed milliseconds per phase to ms_out[LBW_NPHASES] and the number of
 * steps timed to *steps.  Events are host-side runtime objects, pooled in the
 * handle; graph replay is not used while timing. */
int lbw_timing_begin(lbw_handle *h);
int lbw_timing_end(lbw_handle *h, double *ms_out, int64_t *steps);

#ifdef __cplusplus
}
#endif
#endif
