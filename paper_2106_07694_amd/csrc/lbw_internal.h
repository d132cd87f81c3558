// lbw_internal.h -- definitions shared by the HIP translation units of
// liblbw.so (not part of the public ABI; see include/lbw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbw.h"

namespace lbw {

// ---------------------------------------------------------------------------
// Lattices (velocity sets, weights, opposite directions) in the order fixed by
// the public header.  D3Q19 is the lattice of the paper's Fig. 3; D2Q9 is its
// two-dimensional counterpart.  Weights are the standard second-order ones
// (cs^2 = 1/3, eq. 21).
// ---------------------------------------------------------------------------
template <int Q> struct Lattice;

template <> struct Lattice<9> {
    static constexpr int D = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <> struct Lattice<19> {
    static constexpr int D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

// ---------------------------------------------------------------------------
// One run as the kernels see it (passed by value).
// ---------------------------------------------------------------------------
struct RunDev {
    void *f;
    void *c, *c1, *c2;   // C and the two RK stage buffers
    void *s, *s2;        // S and its work buffer (current S is `s`)
    void *u;             // dim*N node velocity
    void *rho;           // N node density, written only when non-NULL
    double *dep;         // per-column deposit
    int32_t nx, ny, nz;  // grid
    int32_t vper;        // vertical axis periodic
    int64_t N;           // nodes
    int64_t ncol;        // bottom columns
    int32_t has_s;
    int32_t scheme;
    int32_t ncls;        // particle size classes: c holds ncls fields of N,
    int32_t pad_;        // dep ncls * ncol counters, class after class
    double tau, omega, guo;          // 1/tau and 1 - 1/(2 tau)
    double body[3], utop[3];
    double vs, kappa_c, gp_c, kappa_s, gp_s, eps;
    double vs_s;         // settling speed Vs (1 - vs_s S) (eq. 13), 0: constant
    double phi_c;        // volume fraction per unit C in the (1 - phi) of eq. 10
};

// Tile shape of the tiled transport kernels for a launch choice.
struct TileShape {
    int tx, ty, chunk;
};

// Arguments of the batched (persistent, work-list) transport launch.  Its
// entries are runs, or size classes of runs (one entry per class, the S
// update carried by the first).
struct BatchArgs {
    const RunDev *runs;        // device copy of the entry table
    const int *tile_start;     // device prefix sum of tiles per entry (nbatch + 1)
    const RunDev *host_runs;   // host copy of the same table
    int nbatch;                // entries
    int chunk;
    int sflip;                 // 1: S and its work buffer are swapped
    int grid;                  // persistent grid size
    int stage = 0;             // 0: the three RK stages and the S update; 1-3: that stage only
    int form = -1;             // -1: every entry; 0 / 1: only the entries with a constant /
                               // S-dependent settling speed (each form in its own kernels)
};

// Launchers (return the launch error, if any).  `odd` selects the second
// kernel of the in-place streaming pair.
hipError_t launch_collide_stream(int q, int precision, const RunDev &r, bool odd,
                                 int block, hipStream_t st);
hipError_t launch_equilibrium(int q, int precision, const RunDev &r, bool odd, const void *rho,
                              const void *u, hipStream_t st);
hipError_t launch_import_f(int q, int precision, const RunDev &r, bool odd, const void *src,
                           hipStream_t st);
hipError_t launch_export_f(int q, int precision, const RunDev &r, bool odd, void *dst,
                           hipStream_t st);
hipError_t launch_transport(int dim, int precision, const RunDev &r, const lbw_launch &l,
                            hipStream_t st);
hipError_t launch_transport_tiled(int dim, int precision, const RunDev &r, const lbw_launch &l,
                                  hipStream_t st);
hipError_t launch_s_update(int dim, int precision, const RunDev &r, hipStream_t st);
// One RK stage (1, 2 or 3) of the tiled transport over the whole grid (runs
// with a constant settling speed).
hipError_t launch_one_stage(int dim, int precision, const RunDev &r, const lbw_launch &l,
                            int stage, hipStream_t st);
TileShape resolve_tile_shape(int dim, const lbw_launch &l);
int64_t transport_tiles(int dim, const RunDev &r, const lbw_launch &l);
hipError_t launch_transport_batched(int dim, int precision, const BatchArgs &b, const lbw_launch &l,
                                    hipStream_t st);
// The tiled stages of runs whose settling speed depends on S (b: batched
// entries, or NULL for the single run r).
hipError_t launch_transport_tiled_vs(int dim, int precision, const RunDev &r, const lbw_launch &l,
                                     hipStream_t st, const BatchArgs *b);
// nodes: total nodes of the batch (chooses the cache policy of the
// population accesses)
hipError_t launch_collide_stream_batched(int q, int precision, const RunDev *runs, const int *blk_start,
                                         int nbatch, int sflip, bool odd, int block, int grid,
                                         int64_t nodes, hipStream_t st);
size_t adjoint_work_bytes(int dim, int precision, int64_t N);
hipError_t launch_adjoint(int q, int precision, const RunDev &r, bool frozen, const void *f_n,
                          const void *c_n, const void *u_n, const void *rho_n, const void *a1_n,
                          const void *a2_n,
                          const void *fbar_next, const void *cbar_next,
                          double dep_bar, void *fbar, void *cbar, double *vs_bar, void *work,
                          const lbw_launch &l, hipStream_t st);
// plane >= 0: MASS_C / MASS_S sum only the cells below that horizontal plane
// (the first plane * ncol nodes of each run); -1: all nodes.  cls >= 0:
// MASS_C and DEPOSIT of that particle size class only; -1: every class.
hipError_t launch_reduce(int q, int precision, const RunDev *runs, int nbatch, int what,
                         bool odd, double *scratch, hipStream_t st, int plane = -1,
                         int cls = -1);
// Power spectral density of a front height (device, ncol values) along
// lateral axis `axis` for slice `index` (-1: mean over slices); out[len/2+1].
hipError_t launch_front_psd(const RunDev &r, int dim, const double *h, int axis, int index,
                            double *out, hipStream_t st);
// Front of the particle field (total over the classes) per bottom column
// into out (device, ncol).
hipError_t launch_front_height(int precision, const RunDev &r, int dim, double thr, double *out,
                               hipStream_t st);

constexpr int kReduceBlocks = 256;  // partial sums per run

}  // namespace lbw
