// transport_tiled.h -- the tiled RK3 stage kernels of the particle
// transport, as templates shared by the two units that build them
// (constant settling speed, and a settling speed set by S).
//
// RK3 stage kernels of the particle transport, tiled for CDNA: a block owns a TX x TY tile of vertical columns and marches up a
// chunk of the vertical axis.  Per plane:
//   * the plane of the stage input a, with a three-cell lateral halo, and the
//     lateral velocities sit in LDS; each lateral face flux is computed once
//     into LDS and differenced by the two cells that share it;
//   * each thread keeps its own column's six-node vertical stencil of a and
//     of the vertical transport velocity in registers, computes the face
//     above its cell and carries it down as the face below the next cell
//     (3D, single precision, WENO5: the stencil's node data instead, each
//     node's flux and indicators computed once, as the node enters);
//   * the next plane's global loads are issued before the current plane is
//     computed (software pipelining).
// Arithmetic and wall rules are those of the plain kernels (transport.hip):
// WENO face fluxes from the upwind side, central diffusion, mirror ghosts
// with a sign flip of the vertical fluid velocity, closed top, absorbing
// bottom feeding the deposit counter.  In single precision the weights use
// the hardware reciprocal.
#pragma once

#include "transport_device.h"

namespace lbw {
namespace {

template <typename T> __device__ __forceinline__ T fast_rcp(T x) { return (T)1 / x; }
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// WENO5-JS face value (the formula of weno5_face) rearranged for issue
// count, with one reciprocal.  The normalised weights are ratios, so every
// indicator may be scaled by one constant and every ideal weight by another:
// with e_k = (12/13)(eps + beta_k) = t_k^2 + (3/13) s_k^2 + (12/13) eps
// (t_k the second difference, s_k the one-sided first difference of
// sub-stencil k, both built from the four first differences) and the
// weights multiplied through by 10 e_0^2 e_1^2 e_2^2, the face value is
//   (P q_0 + Q q_1' + R q_2') / (P + 6 Q + 3 R),
//   P = e_1^2 e_2^2, Q = e_0^2 e_2^2, R = e_0^2 e_1^2,
// where q_0 is the first candidate and q_1' = 6 q_1, q_2' = 3 q_2.
// eps12 is (12/13) eps.  With e_k >= eps12 and concentrations of order one
// every product stays far inside the single-precision range.
template <typename T>
__device__ __forceinline__ T weno5_rcp(T h0, T h1, T h2, T h3, T h4, T a0, T a1, T a2, T a3, T a4,
                                       T eps12) {
    const T g0 = a1 - a0, g1 = a2 - a1, g2 = a3 - a2, g3 = a4 - a3;
    const T t0 = g1 - g0, t1 = g2 - g1, t2 = g3 - g2;
    const T s0 = t0 + (T)2 * g1;          // a0 - 4 a1 + 3 a2
    const T s1 = g1 + g2;                 // a3 - a1
    const T s2 = t2 - (T)2 * g2;          // 3 a2 - 4 a3 + a4
    constexpr T k = (T)(3.0 / 13.0);
    const T e0 = t0 * t0 + (k * s0 * s0 + eps12);
    const T e1 = t1 * t1 + (k * s1 * s1 + eps12);
    const T e2 = t2 * t2 + (k * s2 * s2 + eps12);
    const T S0 = e0 * e0, S1 = e1 * e1, S2 = e2 * e2;
    const T P = S1 * S2, Q = S0 * S2, R = S0 * S1;
    const T q0 = (T)(1.0 / 3.0) * h0 - (T)(7.0 / 6.0) * h1 + (T)(11.0 / 6.0) * h2;
    const T q1 = (T)5 * h2 - h1 + (T)2 * h3;
    const T q2 = h2 + (T)2.5 * h3 - (T)0.5 * h4;
    return (P * q0 + Q * q1 + R * q2) * fast_rcp<T>(P + (T)6 * Q + (T)3 * R);
}

template <typename T>
__device__ __forceinline__ T weno3_rcp(T h0, T h1, T h2, T a0, T a1, T a2, T eps) {
    const T qu = (T)0.5 * ((T)3 * h1 - h0);
    const T qc = (T)0.5 * (h1 + h2);
    const T eu = eps + (a1 - a0) * (a1 - a0);
    const T ec = eps + (a2 - a1) * (a2 - a1);
    const T au = (T)(1.0 / 3.0) * fast_rcp<T>(eu * eu);
    const T ac = (T)(2.0 / 3.0) * fast_rcp<T>(ec * ec);
    return (au * qu + ac * qc) * fast_rcp<T>(au + ac);
}

// Face flux from six nodes j-2..j+3 (a and w given as separate scalars):
// the upwind side is chosen by selects, not branches, so lanes of a wave
// with different face-velocity signs do not diverge.
template <typename T, int SCHEME>
__device__ __forceinline__ T face6(T a0, T a1, T a2, T a3, T a4, T a5, T w0, T w1, T w2, T w3,
                                   T w4, T w5, T kappa, T eps) {
    const bool pos = (w2 + w3) >= (T)0;
    T hh;
    if constexpr (SCHEME == LBW_WENO5) {
        const T A0 = pos ? a0 : a5, A1 = pos ? a1 : a4, A2 = pos ? a2 : a3, A3 = pos ? a3 : a2,
                A4 = pos ? a4 : a1;
        const T W0 = pos ? w0 : w5, W1 = pos ? w1 : w4, W2 = pos ? w2 : w3, W3 = pos ? w3 : w2,
                W4 = pos ? w4 : w1;
        hh = weno5_rcp<T>(W0 * A0, W1 * A1, W2 * A2, W3 * A3, W4 * A4, A0, A1, A2, A3, A4,
                          (T)(12.0 / 13.0) * eps);
    } else if constexpr (SCHEME == LBW_WENO3) {
        const T A0 = pos ? a1 : a4, A1 = pos ? a2 : a3, A2 = pos ? a3 : a2;
        const T W0 = pos ? w1 : w4, W1 = pos ? w2 : w3, W2 = pos ? w3 : w2;
        hh = weno3_rcp<T>(W0 * A0, W1 * A1, W2 * A2, A0, A1, A2, eps);
    } else {
        hh = pos ? w2 * a2 : w3 * a3;
    }
    return hh - kappa * (a3 - a2);
}

// WENO5 with the work of each node done once (the arithmetic of weno5_rcp
// regrouped by node).  Node m is the centre of three sub-stencils that faces
// read: with t = a_{m+1} - 2 a_m + a_{m-1} and c = a_{m+1} - a_{m-1}, their
// scaled indicators are
//   e_c = t^2 + (3/13) c^2 + eps12        (the face's centre sub-stencil),
//   e_l = e_c + (12/13) t (t + c)          (one-sided difference 2t + c, at m+1),
//   e_r = e_c + (12/13) t (t - c)          (one-sided difference 2t - c, at m-1),
// the last two being t^2 + (3/13)(2t +- c)^2 + eps12 expanded (each stays
// within a few units in the last place of its value: e_l, e_r >= t^2 + eps12
// and the cancelling part is at most 2 t^2).  A face takes three of them and
// five node fluxes h = w a, chosen by its upwind side.  Contraction is pinned
// per expression, so every kernel that inlines these gives the same bits.
template <typename T>
__device__ __forceinline__ void weno5_node(T dl, T dr, T eps12, T &el, T &ec, T &er) {
#pragma clang fp contract(on)
    const T t = dr - dl, c = dr + dl;            // dl = a_m - a_{m-1}, dr = a_{m+1} - a_m
    ec = t * t + ((T)(3.0 / 13.0) * c * c + eps12);
    const T kt = (T)(12.0 / 13.0) * t;
    el = kt * (t + c) + ec;
    er = kt * (t - c) + ec;
}

// Total flux through face j+1/2 from node data: fluxes h at j-2 .. j+3, e_l
// at j-1 and j, e_c at j and j+1, e_r at j+1 and j+2, the upwind side (pos:
// the face velocity w_j + w_{j+1} >= 0) and d = a_{j+1} - a_j for diffusion.
// Upwind from j the sub-stencils are centred at j-1 (as the upwind-most), j,
// j+1 (as the downwind-most); upwind from j+1 at j+2, j+1, j, mirrored.
template <typename T>
__device__ __forceinline__ T weno5_flux_nodes(bool pos, T h0, T h1, T h2, T h3, T h4, T h5,
                                              T el_jm1, T el_j, T ec_j, T ec_jp1, T er_jp1,
                                              T er_jp2, T d, T kappa) {
#pragma clang fp contract(on)
    const T H0 = pos ? h0 : h5, H1 = pos ? h1 : h4, H2 = pos ? h2 : h3, H3 = pos ? h3 : h2,
            H4 = pos ? h4 : h1;
    const T e0 = pos ? el_jm1 : er_jp2, e1 = pos ? ec_j : ec_jp1, e2 = pos ? er_jp1 : el_j;
    const T S0 = e0 * e0, S1 = e1 * e1, S2 = e2 * e2;
    const T P = S1 * S2, Q = S0 * S2, R = S0 * S1;
    const T q0 = (T)(1.0 / 3.0) * H0 - (T)(7.0 / 6.0) * H1 + (T)(11.0 / 6.0) * H2;
    const T q1 = (T)5 * H2 - H1 + (T)2 * H3;
    const T q2 = H2 + (T)2.5 * H3 - (T)0.5 * H4;
    const T hh = (P * q0 + Q * q1 + R * q2) * fast_rcp<T>(P + (T)6 * Q + (T)3 * R);
    return hh - kappa * d;
}

struct TileGeom {
    int nx, ny, nv;     // lateral sizes (ny = 1 in 2D) and vertical extent
    int64_t sv;         // stride of the vertical axis
    int64_t N;
    int vper;
    int chunk;          // vertical planes per block
    int gx, gy, gz;     // tiles along x, y and vertical chunks launched
    int bz0;            // first vertical chunk launched
};

// Position of the block: blocks are dealt round-robin to the 8 XCDs, so the
// flat index is remapped to give each XCD a contiguous range of tiles whose
// halos then meet in that XCD's L2.
__device__ __forceinline__ void block_tile(const TileGeom &g, int &bx, int &by, int &bz) {
    const int nb = g.gx * g.gy * g.gz;
    const int b = blockIdx.x;
    int logical = b;
    if ((nb & 7) == 0) {
        const int per = nb >> 3;
        logical = (b & 7) * per + (b >> 3);
    }
    bx = logical % g.gx;
    const int t = logical / g.gx;
    by = t % g.gy;
    bz = g.bz0 + t / g.gy;
}

// Addressing: a vertical plane's base pointer is the same for the whole
// block (uniform, held in scalar registers) and each lane adds a 32-bit byte
// offset within the plane, so the loads and stores need no 64-bit vector
// arithmetic.  This needs nx * ny * sizeof(T) < 2^32 (checked at creation).
template <typename T>
__device__ __forceinline__ const T &at(const void *plane, uint32_t off) {
    return *(const T *)((const char *)plane + off);
}

// FULL: the grid is a whole number of tiles, so every lane owns a cell and
// the store needs no lane mask (a masked store on a path that may be skipped
// would make every later wait on the load counter drain it completely).
// VSS: the settling speed is set by the local fluid density (eq. 13 with rho
// linear in S), Vs (1 - vs_s S) with S at the node (the mirrored node beyond
// a wall); the conservative face fluxes then carry the -phi d(Vs)/dz term of
// eq. 7.  S is read at time level n, which the S update of this step does not
// overwrite (it writes the other S buffer).
// FS (stage 1 only): the S update (S5-S6 in conservative form, the
// arithmetic and sum order of k_s_update) rides with the march.  It needs the
// velocity this stage already stages (lateral components in LDS, the
// vertical one read per plane) plus S on the plane with a one-cell lateral
// halo and at the next plane of the column; s_entry is false for a batch
// entry that carries no S (a size class after the first), which then loads
// C in its place and stores nothing.
template <typename T, int D, int SCHEME, int STAGE, int TX, int TY, bool FULL, bool VSS,
          bool FS = false>
__device__ __forceinline__ void stage_tile(const RunDev &r, const TileGeom &g, int bx, int by, int bz,
                                           bool s_entry = true) {
    static_assert(!FS || STAGE == 1, "the S update rides with stage 1");
    constexpr int NT = TX * TY;
    constexpr int AX = TX + 6;                  // a plane row length (x halo 3 + 3)
    constexpr int AY = (D == 3) ? TY + 6 : 1;   // a plane rows
    // NV (3D, single precision, WENO5): the vertical faces share each node's
    // work (its flux w a and the three indicators it centres, weno5_node),
    // done once as the node enters the column's window; the fluxes and
    // differences stay in registers, the indicators in a per-thread LDS ring
    // (in registers they would cost a block of occupancy).  The lateral faces
    // keep face6: shared node data there needs an extra LDS round trip and
    // barrier per plane, which cost more than the arithmetic saves, and 2D
    // tiles wait on their barriers and loads rather than on instruction issue.
    constexpr bool NV = (SCHEME == LBW_WENO5 && D == 3 && sizeof(T) == 4);
    constexpr int SXL = TX + 2;                         // S row with a one-cell x halo
    constexpr int SYL = (D == 3) ? TY + 2 : 1;          // S rows (one-cell y halo in 3D)
    // The LDS arrays are pieces of one allocation at fixed offsets, so that
    // accesses which share a lane-dependent index can share one address
    // register and differ only in the instruction's constant offset.
    constexpr int O_A = 0, O_UX = AY * AX, O_UY = O_UX + TY * AX,
                  O_FX = O_UY + ((D == 3) ? (TY + 6) * TX : 1), O_FY = O_FX + TY * (TX + 1),
                  O_S = O_FY + ((D == 3) ? (TY + 1) * TX : 1), O_GX = O_S + (FS ? SXL * SYL : 1),
                  O_GY = O_GX + (FS ? TY * (TX + 1) : 1),
                  O_END = O_GY + ((FS && D == 3) ? (TY + 1) * TX : 1);
    __shared__ T smem[O_END];
    T *const sA = smem + O_A;                   // stage input a, plane with halos
    T *const sUx = smem + O_UX;                 // x velocity, rows with x halo
    T *const sUy = smem + O_UY;                 // y velocity, columns with y halo
    T *const sFx = smem + O_FX;                 // x face fluxes
    T *const sFy = smem + O_FY;                 // y face fluxes
    T *const sS = smem + O_S;                   // S plane with a one-cell halo
    T *const sGx = smem + O_GX;                 // S face fluxes
    T *const sGy = smem + O_GY;

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = bx * TX, y0 = by * TY;
    const int gxl = x0 + tx, gyl = y0 + ty;         // own column (may be outside)
    const bool active = FULL || (gxl < g.nx && (D == 2 || gyl < g.ny));
    const int xw = active ? gxl : gxl % g.nx;       // wrapped column for loads
    const int yw = (D == 3) ? (active ? gyl : gyl % g.ny) : 0;
    const int col = xw + g.nx * yw;                 // < nx * ny
    uint32_t colb = (uint32_t)col * (uint32_t)sizeof(T);
    const int v0 = bz * g.chunk;
    const int v1 = min(v0 + g.chunk, g.nv);

    const T *__restrict__ ain = (const T *)(STAGE == 1 ? r.c : (STAGE == 2 ? r.c1 : r.c2));
    const T *__restrict__ ux = (const T *)r.u;
    const T *__restrict__ uy = ux + g.N;
    const T *__restrict__ uv = ux + (int64_t)(D - 1) * g.N;
    const T vs = (T)r.vs, kap = (T)r.kappa_c, eps = (T)r.eps;
    const bool walls = !g.vper;
    auto plane = [&](const void *base, int v) -> const void * {
        return (const char *)base + (int64_t)v * g.sv * (int64_t)sizeof(T);
    };
    // settling speed at plane vv of this column
    auto vs_at = [&](int vv) -> T {
        if constexpr (VSS) return vs * ((T)1 - (T)r.vs_s * at<T>(plane(r.s, vv), colb));
        else return vs;
    };
    auto wplane = [&](void *base, int v) -> void * {
        return (char *)base + (int64_t)v * g.sv * (int64_t)sizeof(T);
    };

    // vertical index with the wall/periodic rule; sets flip for mirrored nodes
    auto vidx = [&](int v, bool &flip) -> int {
        flip = false;
        // the march reaches at most three planes below and four above the
        // axis (v in [-3, nv + 3]) and nv >= 6, so one wrap suffices
        if (!walls) return v < 0 ? v + g.nv : (v >= g.nv ? v - g.nv : v);
        if (v < 0) { flip = true; return -1 - v; }
        if (v >= g.nv) { flip = true; return 2 * g.nv - 1 - v; }
        return v;
    };
    auto load_av = [&](int v, T &a, T &w) {
        bool flip;
        const int vv = vidx(v, flip);
        a = at<T>(plane(ain, vv), colb);
        const T u = at<T>(plane(uv, vv), colb);
        w = (flip ? -u : u) - vs_at(vv);
    };

    // lateral halo slots of this thread (fixed over the march), as byte
    // offsets within a plane and LDS indices (-1: no slot)
    // a-plane cross: rows ty in [0,TY) x cols [0,AX), plus (3D) y-halo rows
    constexpr int NA = (D == 3) ? AX * TY + TX * 6 : AX;
    constexpr int NUX = AX * TY;
    constexpr int NUY = (D == 3) ? TX * (TY + 6) : 0;
    constexpr int SA = (NA + NT - 1) / NT, SUX = (NUX + NT - 1) / NT, SUY = (NUY + NT - 1) / NT;
    uint32_t offA[SA];
    int ldsA[SA];
    uint32_t offX[SUX];
    int ldsX[SUX];
    uint32_t offY[(SUY > 0) ? SUY : 1];
    int ldsY[(SUY > 0) ? SUY : 1];
    auto wrapx = [&](int x) { x %= g.nx; return x < 0 ? x + g.nx : x; };
    auto wrapy = [&](int y) { y %= g.ny; return y < 0 ? y + g.ny : y; };
    auto lat = [&](int x, int y) { return (uint32_t)(x + g.nx * y) * (uint32_t)sizeof(T); };
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        const int i = tid + s * NT;
        ldsA[s] = -1;
        offA[s] = 0;
        if (i < NA) {
            int lx, ly;  // plane-local coords, halo origin at (-3, -3)
            if (i < AX * TY) { lx = i % AX; ly = (D == 3) ? (i / AX) + 3 : 0; }
            else { const int j = i - AX * TY; lx = (j % TX) + 3; ly = (j / TX) < 3 ? (j / TX) : (j / TX) + TY; }
            offA[s] = lat(wrapx(x0 + lx - 3), (D == 3) ? wrapy(y0 + ly - 3) : 0);
            ldsA[s] = ly * AX + lx;
        }
    }
#pragma unroll
    for (int s = 0; s < SUX; ++s) {
        const int i = tid + s * NT;
        ldsX[s] = -1;
        offX[s] = 0;
        if (i < NUX) {
            const int lx = i % AX, ly = i / AX;
            offX[s] = lat(wrapx(x0 + lx - 3), (D == 3) ? wrapy(y0 + ly) : 0);
            ldsX[s] = ly * AX + lx;
        }
    }
#pragma unroll
    for (int s = 0; s < SUY; ++s) {
        const int i = tid + s * NT;
        ldsY[s] = -1;
        offY[s] = 0;
        if (i < NUY) {
            const int lx = i % TX, ly = i / TX;
            offY[s] = lat(wrapx(x0 + lx), wrapy(y0 + ly - 3));
            ldsY[s] = ly * TX + lx;
        }
    }

    // S slots (FS): the plane's S on the tile with a one-cell halo (the 3D
    // corners are loaded and not read)
    constexpr int NSS = FS ? SXL * SYL : 0;
    constexpr int SSS = (NSS + NT - 1) / NT;
    uint32_t offS[(SSS > 0) ? SSS : 1];
    int ldsS[(SSS > 0) ? SSS : 1];
#pragma unroll
    for (int s = 0; s < SSS; ++s) {
        const int i = tid + s * NT;
        ldsS[s] = -1;
        offS[s] = 0;
        if (i < NSS) {
            const int lx = i % SXL, ly = i / SXL;
            offS[s] = lat(wrapx(x0 + lx - 1), (D == 3) ? wrapy(y0 + ly - 1) : 0);
            ldsS[s] = i;
        }
    }
    const T *__restrict__ sin = (const T *)(FS && s_entry ? r.s : r.c);
    const T kaps = (T)r.kappa_s;
    // S face between nodes j (a2, w2) and j + 1 (a3, w3)
    auto sface = [&](T a2, T a3, T w2, T w3) -> T {
        const T hh = ((T)0.5 * (w2 + w3) >= (T)0) ? w2 * a2 : w3 * a3;
        return hh - kaps * (a3 - a2);
    };

    constexpr int NEX = (D == 3) ? TX + TY : 1;   // faces on the tile's far edges

    // vertical windows for the face above v: a and w at v-2 .. v+3 (face6),
    // or (NV) the node data of the same nodes: fluxes vH at v-2 .. v+3, the
    // indicators e_l, e_c, e_r of nodes v-1 .. v+2 (EL, EC, ER), and for the
    // faces j+1/2, j = v .. v+2, the upwind side vP (w_j + w_{j+1} >= 0) and
    // the difference vD = a_{j+1} - a_j (a face's slot is its lower node's);
    // a_last, w_last hold node v+3
    const T eps12 = (T)(12.0 / 13.0) * eps;
    T aw[6], ww[6];
    T vH[6], vD[6];
    // the indicators of the window's nodes, per thread in LDS (six-slot rings
    // that rotate like the window; each thread reads only what it wrote)
    __shared__ T sE[NV ? 18 * NT : 1];
    auto EL = [&](int slot) -> T & { return sE[(0 * 6 + slot) * NT + tid]; };
    auto EC = [&](int slot) -> T & { return sE[(1 * 6 + slot) * NT + tid]; };
    auto ER = [&](int slot) -> T & { return sE[(2 * 6 + slot) * NT + tid]; };
    bool vP[6];
    T a_last = (T)0, w_last = (T)0, a_first;
    T fbelow;                                       // face below the first plane
    if constexpr (NV) {
        T an[7], wn[7], hn[7], dn[6], sn[6], ln[7], cn[7], rn[7];   // nodes v0-3 .. v0+3
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            load_av(v0 - 3 + k, an[k], wn[k]);
            hn[k] = wn[k] * an[k];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            dn[k] = an[k + 1] - an[k];
            sn[k] = wn[k] + wn[k + 1];
        }
#pragma unroll
        for (int k = 1; k < 6; ++k) weno5_node<T>(dn[k - 1], dn[k], eps12, ln[k], cn[k], rn[k]);
        // window position m is node v0-2+m, index k = m+1 here
#pragma unroll
        for (int m = 0; m < 6; ++m) vH[m] = hn[m + 1];
#pragma unroll
        for (int m = 1; m < 5; ++m) {
            EL(m) = ln[m + 1];
            EC(m) = cn[m + 1];
            ER(m) = rn[m + 1];
        }
#pragma unroll
        for (int m = 2; m < 5; ++m) {
            vP[m] = sn[m + 1] >= (T)0;
            vD[m] = dn[m + 1];
        }
        a_last = an[6];
        w_last = wn[6];
        a_first = an[3];
        if (!(walls && v0 == 0))
            fbelow = weno5_flux_nodes<T>(sn[2] >= (T)0, hn[0], hn[1], hn[2], hn[3], hn[4], hn[5], ln[1],
                                         ln[2], cn[2], cn[3], rn[3], rn[4], dn[2], kap);
    } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) load_av(v0 - 2 + m, aw[m], ww[m]);
        a_first = aw[2];
        if (!(walls && v0 == 0)) {
            T ab, wb;
            load_av(v0 - 3, ab, wb);
            fbelow = face6<T, SCHEME>(ab, aw[0], aw[1], aw[2], aw[3], aw[4], wb, ww[0], ww[1], ww[2],
                                      ww[3], ww[4], kap, eps);
        }
    }
    if (walls && v0 == 0) fbelow = -vs_at(0) * a_first;   // absorbing bottom

    // S and the raw vertical velocity at this plane of the column, and the S
    // face below the first plane (closed walls; periodic: wrapped)
    T s_c = (T)0, us_c = (T)0, gbelow = (T)0;
    if constexpr (FS) {
        s_c = at<T>(plane(sin, v0), colb);
        us_c = at<T>(plane(uv, v0), colb);
        if (!(walls && v0 == 0)) {
            bool flip;
            const int vb = vidx(v0 - 1, flip);
            gbelow = sface(at<T>(plane(sin, vb), colb), s_c, at<T>(plane(uv, vb), colb), us_c);
        }
    }

    // deposit of stage 3 (D += Vs (C/6 + a1/6 + 2 a2/3) at the bottom cell),
    // done before the march so that no load or store sits on a path of its own
    if constexpr (STAGE == 3) {
        if (walls && v0 == 0 && active) {
            // the deposit's settling speed in FP64 (vs_s = 0: exactly vs)
            const double vsd =
                VSS ? r.vs * (1.0 - r.vs_s * (double)at<T>(plane(r.s, 0), colb)) : r.vs;
            const double o0 = vsd * (double)at<T>(plane(r.c, 0), colb);
            const double o1 = vsd * (double)at<T>(plane(r.c1, 0), colb);
            const double o2 = vsd * (double)a_first;
            r.dep[col] += o0 / 6.0 + o1 / 6.0 + 2.0 / 3.0 * o2;
        }
    }

    // prefetch registers for the lateral planes
    T pA[SA], pX[SUX], pY[(SUY > 0) ? SUY : 1], pS[(SSS > 0) ? SSS : 1];
    auto prefetch = [&](int v) {
        bool flip;
        const int vv = vidx(v, flip);
        const void *pa = plane(ain, vv), *px = plane(ux, vv), *py = plane(uy, vv);
#pragma unroll
        for (int s = 0; s < SSS; ++s) pS[s] = at<T>(plane(sin, vv), offS[s]);
        // unconditional: slots without an LDS target read column 0 (in
        // bounds) and are dropped at publication, so no load sits behind a
        // branch
#pragma unroll
        for (int s = 0; s < SA; ++s) pA[s] = at<T>(pa, offA[s]);
#pragma unroll
        for (int s = 0; s < SUX; ++s) pX[s] = at<T>(px, offX[s]);
#pragma unroll
        for (int s = 0; s < SUY; ++s) pY[s] = at<T>(py, offY[s]);
    };
    prefetch(v0);

    // The march is unrolled six planes at a time with the window slots
    // rotating: at phase ph, window position m lives in slot (ph + m) % 6,
    // and the node entering at v + 4 takes the slot position 0 leaves, so no
    // register moves shift the window from plane to plane.
    for (int vb = v0; vb < v1; vb += 6) {
#pragma unroll
        for (int ph = 0; ph < 6; ++ph) {
            const int v = vb + ph;
            if (v >= v1) break;
            // window position m (node v - 2 + m) of this phase
            auto A = [&](int m) -> T & { return aw[(ph + m) % 6]; };
            auto W = [&](int m) -> T & { return ww[(ph + m) % 6]; };
            // the lane offsets pass through an empty asm every plane: the
            // compiler can then no longer fold them into per-lane 64-bit
            // pointers hoisted out of the march (each plane's offset would be
            // added to those in vector instructions), and the loads keep the
            // scalar-base plus 32-bit-offset form
            asm volatile("" : "+v"(colb));
#pragma unroll
            for (int s = 0; s < SA; ++s) asm volatile("" : "+v"(offA[s]));
#pragma unroll
            for (int s = 0; s < SUX; ++s) asm volatile("" : "+v"(offX[s]));
#pragma unroll
            for (int s = 0; s < SUY; ++s) asm volatile("" : "+v"(offY[s]));
#pragma unroll
            for (int s = 0; s < SSS; ++s) asm volatile("" : "+v"(offS[s]));
            // publish plane v
#pragma unroll
            for (int s = 0; s < SA; ++s) if (ldsA[s] >= 0) sA[ldsA[s]] = pA[s];
#pragma unroll
            for (int s = 0; s < SUX; ++s) if (ldsX[s] >= 0) sUx[ldsX[s]] = pX[s];
#pragma unroll
            for (int s = 0; s < SUY; ++s) if (ldsY[s] >= 0) sUy[ldsY[s]] = pY[s];
#pragma unroll
            for (int s = 0; s < SSS; ++s) if (ldsS[s] >= 0) sS[ldsS[s]] = pS[s];
            __syncthreads();
            // loads, in the order they are consumed (the load counter drains in
            // issue order, so waiting for one waits for all issued before it):
            // this cell's C and the vertical pair at v+4, both used at the end of
            // this plane, then the next lateral plane, used only after the next
            // barrier and so in flight across this plane's face computation
            // (past the chunk it is still a valid plane: the vertical rule maps
            // it inside)
            T cown = (T)0;
            if (STAGE != 1) cown = at<T>(plane(r.c, v), colb);
            T anext, wnext;
            load_av(v + 4, anext, wnext);
            T s_n = (T)0, us_n = (T)0;
            if constexpr (FS) {
                bool flip;
                const int vn = vidx(v + 1, flip);
                s_n = at<T>(plane(sin, vn), colb);
                us_n = at<T>(plane(uv, vn), colb);
            }
            prefetch(v + 1);

            // each thread the x face on the left of its cell and (3D) the y
            // face below it; the stage input at the cell is the x stencil's
            // fourth node
            T a_own;
            {
                const T *ar = sA + ((D == 3) ? (ty + 3) : 0) * AX + tx;   // nodes tx-3 .. tx+2
                const T *ur = sUx + ty * AX + tx;
                sFx[ty * (TX + 1) + tx] = face6<T, SCHEME>(ar[0], ar[1], ar[2], ar[3], ar[4], ar[5], ur[0],
                                                            ur[1], ur[2], ur[3], ur[4], ur[5], kap, eps);
                a_own = ar[3];
            }
            if constexpr (D == 3) {
                const T *ac = sA + ty * AX + tx + 3;      // rows ty-3+3 .. ty+2+3 of column tx
                const T *uc = sUy + ty * TX + tx;
                sFy[ty * TX + tx] = face6<T, SCHEME>(ac[0], ac[AX], ac[2 * AX], ac[3 * AX], ac[4 * AX],
                                                     ac[5 * AX], uc[0], uc[TX], uc[2 * TX], uc[3 * TX],
                                                     uc[4 * TX], uc[5 * TX], kap, eps);
            }
            if constexpr (FS) {
                // S faces on the left of the cell and (3D) below it
                const T *sr = sS + ((D == 3) ? ty + 1 : 0) * SXL + tx;     // x - 1, x
                const T *ur = sUx + ty * AX + tx + 2;
                sGx[ty * (TX + 1) + tx] = sface(sr[0], sr[1], ur[0], ur[1]);
                if constexpr (D == 3) {
                    const T *sc = sS + ty * SXL + tx + 1;                  // y - 1, y
                    const T *uc = sUy + (ty + 2) * TX + tx;
                    sGy[ty * TX + tx] = sface(sc[0], sc[SXL], uc[0], uc[TX]);
                }
            }
            // faces on the far edges of the tile, taken by the first lanes in
            // one extra pass, so that the main passes are exactly one face
            // per thread: (3D) the y faces of row TY first, so that they
            // fill whole waves (a lane with tid < TX has ty = 0 and tx = tid,
            // so their addresses are the main pass's plus a constant), then
            // the x faces of column TX
            static_assert(NEX <= NT, "one pass of edge faces");
            if (D == 3 && tid < TX) {
                if constexpr (D == 3) {
                    const T *ac = sA + (ty + TY) * AX + tx + 3;
                    const T *uc = sUy + (ty + TY) * TX + tx;
                    sFy[(ty + TY) * TX + tx] = face6<T, SCHEME>(ac[0], ac[AX], ac[2 * AX], ac[3 * AX],
                                                                ac[4 * AX], ac[5 * AX], uc[0], uc[TX],
                                                                uc[2 * TX], uc[3 * TX], uc[4 * TX],
                                                                uc[5 * TX], kap, eps);
                    if constexpr (FS) {
                        const T *sc = sS + (ty + TY) * SXL + tx + 1;
                        const T *uc2 = sUy + (ty + TY + 2) * TX + tx;
                        sGy[(ty + TY) * TX + tx] = sface(sc[0], sc[SXL], uc2[0], uc2[TX]);
                    }
                }
            } else if (tid < NEX) {
                const int fy = tid - ((D == 3) ? TX : 0);
                const T *ar = sA + ((D == 3) ? (fy + 3) : 0) * AX + TX;
                const T *ur = sUx + fy * AX + TX;
                sFx[fy * (TX + 1) + TX] = face6<T, SCHEME>(ar[0], ar[1], ar[2], ar[3], ar[4], ar[5], ur[0],
                                                           ur[1], ur[2], ur[3], ur[4], ur[5], kap, eps);
                if constexpr (FS) {
                    const T *sr = sS + ((D == 3) ? fy + 1 : 0) * SXL + TX;
                    const T *ur2 = sUx + fy * AX + TX + 2;
                    sGx[fy * (TX + 1) + TX] = sface(sr[0], sr[1], ur2[0], ur2[1]);
                }
            }
            // vertical face above this cell
            T fabove;
            if (walls && v == g.nv - 1) {
                fabove = (T)0;
            } else if constexpr (NV) {
                auto S6 = [&](int m) { return (ph + m) % 6; };
                fabove = weno5_flux_nodes<T>(vP[S6(2)], vH[S6(0)], vH[S6(1)], vH[S6(2)],
                                             vH[S6(3)], vH[S6(4)], vH[S6(5)], EL(S6(1)), EL(S6(2)),
                                             EC(S6(2)), EC(S6(3)), ER(S6(3)), ER(S6(4)), vD[S6(2)], kap);
            } else {
                fabove = face6<T, SCHEME>(A(0), A(1), A(2), A(3), A(4), A(5), W(0), W(1), W(2), W(3),
                                          W(4), W(5), kap, eps);
            }
            T gabove = (T)0;
            if constexpr (FS) gabove = (walls && v == g.nv - 1) ? (T)0 : sface(s_c, s_n, us_c, us_n);
            __syncthreads();
            T L = -(fabove - fbelow);
            L -= sFx[ty * (TX + 1) + tx + 1] - sFx[ty * (TX + 1) + tx];
            if constexpr (D == 3) L -= sFy[(ty + 1) * TX + tx] - sFy[ty * TX + tx];
            const T a = a_own;
            if (active) {
                if constexpr (STAGE == 1) {
                    *(T *)((char *)wplane(r.c1, v) + colb) = a + L;
                } else if constexpr (STAGE == 2) {
                    *(T *)((char *)wplane(r.c2, v) + colb) = rk3_stage2<T>(cown, a, L);
                } else {
                    *(T *)((char *)wplane(r.c, v) + colb) = rk3_stage3<T>(cown, a, L);
                }
            }
            if constexpr (FS) {
                T Ls = -(sGx[ty * (TX + 1) + tx + 1] - sGx[ty * (TX + 1) + tx]);
                if constexpr (D == 3) Ls -= sGy[(ty + 1) * TX + tx] - sGy[ty * TX + tx];
                Ls -= gabove - gbelow;
                if (active && s_entry) *(T *)((char *)wplane(r.s2, v) + colb) = s_c + Ls;
                gbelow = gabove;
                s_c = s_n;
                us_c = us_n;
            }
            fbelow = fabove;
            // node v + 4 enters, position 0 leaves
            if constexpr (NV) {
                const T dnew = anext - a_last;
                T el, ec, er;
                weno5_node<T>(vD[(ph + 4) % 6], dnew, eps12, el, ec, er);
                EL((ph + 5) % 6) = el;
                EC((ph + 5) % 6) = ec;
                ER((ph + 5) % 6) = er;
                vD[(ph + 5) % 6] = dnew;
                vP[(ph + 5) % 6] = (w_last + wnext) >= (T)0;
                vH[ph % 6] = wnext * anext;
                a_last = anext;
                w_last = wnext;
            } else {
                A(0) = anext;
                W(0) = wnext;
            }
            // no barrier here: the next plane's publication writes arrays
            // last read before the barrier above, and the face arrays read
            // since are next written after that plane's own first barrier
        }
    }
}

template <typename T, int D, int SCHEME, int STAGE, int TX, int TY, bool FULL, bool VSS, bool FS = false>
__global__ void __launch_bounds__(TX *TY) k_stage_tiled(RunDev r, TileGeom g) {
    int bx, by, bz;
    block_tile(g, bx, by, bz);
    stage_tile<T, D, SCHEME, STAGE, TX, TY, FULL, VSS, FS>(r, g, bx, by, bz, true);
}

template <int D>
__host__ __device__ inline TileGeom make_geom(const RunDev &r, int chunk, int TX, int TY) {
    TileGeom g;
    g.nx = r.nx;
    g.ny = (D == 3) ? r.ny : 1;
    g.nv = (D == 3) ? r.nz : r.ny;
    g.sv = (D == 3) ? (int64_t)r.nx * r.ny : (int64_t)r.nx;
    g.N = r.N;
    g.vper = r.vper;
    g.chunk = chunk < g.nv ? chunk : g.nv;
    g.gx = (r.nx + TX - 1) / TX;
    g.gy = (D == 3) ? (r.ny + TY - 1) / TY : 1;
    g.gz = (g.nv + g.chunk - 1) / g.chunk;
    g.bz0 = 0;
    return g;
}

// Batched form: one persistent grid walks the tiles of every run.  Each XCD
// takes a contiguous range of the global tile list (runs in order, tiles of
// a run x-fastest), so neighbouring tiles share an L2.  tile_start[b] is the
// first global tile of run b (prefix sum, nbatch + 1 entries).
template <typename T, int D, int SCHEME, int STAGE, int TX, int TY, bool VSS, bool FS = false>
__global__ void __launch_bounds__(TX *TY) k_stage_batched(const RunDev *__restrict__ runs,
                                                          const int *__restrict__ tile_start,
                                                          int nbatch, int chunk, int sflip,
                                                          int form) {
    const int total = tile_start[nbatch];
    const int G = gridDim.x;
    // with 8 blocks or more, block i runs on XCD i % 8 and that XCD walks its
    // own contiguous range; a smaller grid would leave some ranges with no
    // block, so it walks the whole list instead
    int first = blockIdx.x, stride = G, hi = total;
    if (G >= 8) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        const int per_xcd = (G + 7 - xcd) >> 3;           // blocks on this XCD (>= 1)
        first = (int)((int64_t)total * xcd / 8) + slot;
        hi = (int)((int64_t)total * (xcd + 1) / 8);
        stride = per_xcd;
    }
    for (int w = first; w < hi; w += stride) {
        int b = 0;
        while (tile_start[b + 1] <= w) ++b;                // runs are few; linear scan
        RunDev r = runs[b];
        if (form >= 0 && (r.vs_s != 0.0) != (form == 1)) continue;   // the other form's entry
        if (sflip) { void *t = r.s; r.s = r.s2; r.s2 = t; }
        const TileGeom g = make_geom<D>(r, chunk, TX, TY);
        const int t = w - tile_start[b];
        const int bx = t % g.gx, rest = t / g.gx;
        stage_tile<T, D, SCHEME, STAGE, TX, TY, false, VSS, FS>(r, g, bx, rest % g.gy, rest / g.gy,
                                                               r.has_s != 0);
    }
}

// The whole-tile form when the grid divides into tiles, else the masked one
// (runs with a variable settling speed always take the masked form, which
// halves the kernels built for them).
template <typename T, int D, int SCHEME, int STAGE, int TX, int TY, bool VSS, bool FS = false>
void launch_stage(const RunDev &r, const TileGeom &g, unsigned nb, hipStream_t st) {
    if constexpr (!VSS) {
        if (g.nx % TX == 0 && (D == 2 || g.ny % TY == 0)) {
            k_stage_tiled<T, D, SCHEME, STAGE, TX, TY, true, false, FS><<<nb, TX * TY, 0, st>>>(r, g);
            return;
        }
    }
    k_stage_tiled<T, D, SCHEME, STAGE, TX, TY, false, VSS, FS><<<nb, TX * TY, 0, st>>>(r, g);
}

// Stage 1, carrying the S update when the run has S.
template <typename T, int D, int SCHEME, int TX, int TY, bool VSS>
void launch_stage1(const RunDev &r, const TileGeom &g, unsigned nb, hipStream_t st) {
    if (r.has_s) launch_stage<T, D, SCHEME, 1, TX, TY, VSS, true>(r, g, nb, st);
    else launch_stage<T, D, SCHEME, 1, TX, TY, VSS, false>(r, g, nb, st);
}

template <typename T, int D, int SCHEME, int TX, int TY, bool VSS>
hipError_t stages(const RunDev &r, int chunk, hipStream_t st) {
    const TileGeom g = make_geom<D>(r, chunk, TX, TY);
    const int64_t nb = (int64_t)g.gx * g.gy * g.gz;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    launch_stage1<T, D, SCHEME, TX, TY, VSS>(r, g, (unsigned)nb, st);
    launch_stage<T, D, SCHEME, 2, TX, TY, VSS>(r, g, (unsigned)nb, st);
    launch_stage<T, D, SCHEME, 3, TX, TY, VSS>(r, g, (unsigned)nb, st);
    return hipGetLastError();
}

template <typename T, int D, int SCHEME, int TX, int TY>
hipError_t one_stage_t(const RunDev &r, int chunk, int stage, hipStream_t st) {
    const TileGeom g = make_geom<D>(r, chunk, TX, TY);
    const int64_t nb = (int64_t)g.gx * g.gy * g.gz;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (stage == 1) launch_stage1<T, D, SCHEME, TX, TY, false>(r, g, (unsigned)nb, st);
    else if (stage == 2) launch_stage<T, D, SCHEME, 2, TX, TY, false>(r, g, (unsigned)nb, st);
    else launch_stage<T, D, SCHEME, 3, TX, TY, false>(r, g, (unsigned)nb, st);
    return hipGetLastError();
}

// Calls fn(integral_constant TX, integral_constant TY) for the tile shape:
// 3D 32x8, 64x4, 128x2 (256 threads), 32x16, 64x8 (512 threads); 2D one row
// of 64, 128, 256 or 512 columns.
template <int D, typename F>
hipError_t with_tile(const TileShape &sh, F &&fn) {
    using std::integral_constant;
    if constexpr (D == 3) {
        if (sh.tx == 64 && sh.ty == 8) return fn(integral_constant<int, 64>{}, integral_constant<int, 8>{});
        if (sh.tx == 32 && sh.ty == 16) return fn(integral_constant<int, 32>{}, integral_constant<int, 16>{});
        if (sh.tx == 64) return fn(integral_constant<int, 64>{}, integral_constant<int, 4>{});
        if (sh.tx == 128) return fn(integral_constant<int, 128>{}, integral_constant<int, 2>{});
        return fn(integral_constant<int, 32>{}, integral_constant<int, 8>{});
    } else {
        if (sh.tx == 64) return fn(integral_constant<int, 64>{}, integral_constant<int, 1>{});
        if (sh.tx == 128) return fn(integral_constant<int, 128>{}, integral_constant<int, 1>{});
        if (sh.tx == 512) return fn(integral_constant<int, 512>{}, integral_constant<int, 1>{});
        return fn(integral_constant<int, 256>{}, integral_constant<int, 1>{});
    }
}

template <typename T, int D, int SCHEME>
hipError_t one_stage_shape(const RunDev &r, const lbw_launch &l, int stage, hipStream_t st) {
    const TileShape sh = resolve_tile_shape(D, l);
    return with_tile<D>(sh, [&](auto tx, auto ty) {
        return one_stage_t<T, D, SCHEME, decltype(tx)::value, decltype(ty)::value>(r, sh.chunk, stage, st);
    });
}

template <typename T, int D>
hipError_t one_stage_d(const RunDev &r, const lbw_launch &l, int stage, hipStream_t st) {
    switch (r.scheme) {
        case LBW_WENO5: return one_stage_shape<T, D, LBW_WENO5>(r, l, stage, st);
        case LBW_WENO3: return one_stage_shape<T, D, LBW_WENO3>(r, l, stage, st);
        case LBW_UPWIND1: return one_stage_shape<T, D, LBW_UPWIND1>(r, l, stage, st);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D, int SCHEME, int TX, int TY, bool VSS>
hipError_t stages_batched(const BatchArgs &a, hipStream_t st) {
    bool any_s = false;
    for (int i = 0; i < a.nbatch; ++i) any_s = any_s || a.host_runs[i].has_s;
    auto stage = [&](int k) {
        if (k == 1 && any_s)
            k_stage_batched<T, D, SCHEME, 1, TX, TY, VSS, true><<<a.grid, TX * TY, 0, st>>>(
                a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip, a.form);
        else if (k == 1)
            k_stage_batched<T, D, SCHEME, 1, TX, TY, VSS><<<a.grid, TX * TY, 0, st>>>(
                a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip, a.form);
        else if (k == 2)
            k_stage_batched<T, D, SCHEME, 2, TX, TY, VSS><<<a.grid, TX * TY, 0, st>>>(
                a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip, a.form);
        else
            k_stage_batched<T, D, SCHEME, 3, TX, TY, VSS><<<a.grid, TX * TY, 0, st>>>(
                a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip, a.form);
        return hipGetLastError();
    };
    if (a.stage != 0) return stage(a.stage);
    hipError_t e = stage(1);
    if (e == hipSuccess) e = stage(2);
    if (e == hipSuccess) e = stage(3);
    return e;
}

template <typename T, int D, int SCHEME, bool VSS>
hipError_t stages_shape(const RunDev &r, const lbw_launch &l, hipStream_t st, const BatchArgs *batch) {
    const TileShape sh = resolve_tile_shape(D, l);
    return with_tile<D>(sh, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        return batch ? stages_batched<T, D, SCHEME, TX, TY, VSS>(*batch, st)
                     : stages<T, D, SCHEME, TX, TY, VSS>(r, sh.chunk, st);
    });
}

template <typename T, int D, bool VSS>
hipError_t tiled_d(const RunDev &r, const lbw_launch &l, hipStream_t st, const BatchArgs *b) {
    switch (r.scheme) {
        case LBW_WENO5: return stages_shape<T, D, LBW_WENO5, VSS>(r, l, st, b);
        case LBW_WENO3: return stages_shape<T, D, LBW_WENO3, VSS>(r, l, st, b);
        case LBW_UPWIND1: return stages_shape<T, D, LBW_UPWIND1, VSS>(r, l, st, b);
    }
    return hipErrorInvalidValue;
}

// Both precisions and dimensions for one settling form.
template <bool VSS>
hipError_t tiled_any(int dim, int precision, const RunDev &r, const lbw_launch &l, hipStream_t st,
                     const BatchArgs *b) {
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? tiled_d<float, 2, VSS>(r, l, st, b) : tiled_d<float, 3, VSS>(r, l, st, b);
    return dim == 2 ? tiled_d<double, 2, VSS>(r, l, st, b) : tiled_d<double, 3, VSS>(r, l, st, b);
}

}  // namespace
}  // namespace lbw
