// transport_tiled.hip -- RK3 stage kernels of the particle transport, tiled
// for CDNA: a block owns a TX x TY tile of vertical columns and marches up a
// chunk of the vertical axis.  Per plane:
//   * the plane of the stage input a, with a three-cell lateral halo, and the
//     lateral velocities sit in LDS; each lateral face flux is computed once
//     into LDS and differenced by the two cells that share it;
//   * each thread keeps its own column's six-node vertical stencil of a and
//     of the vertical transport velocity in registers, computes the face
//     above its cell and carries it down as the face below the next cell;
//   * the next plane's global loads are issued before the current plane is
//     computed (software pipelining).
// Arithmetic and wall rules are those of the plain kernels (transport.hip):
// WENO face fluxes from the upwind side, central diffusion, mirror ghosts
// with a sign flip of the vertical fluid velocity, closed top, absorbing
// bottom feeding the deposit counter.  In single precision the weights use
// the hardware reciprocal.
#include "transport_device.h"

namespace lbw {
namespace {

template <typename T> __device__ __forceinline__ T fast_rcp(T x) { return (T)1 / x; }
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// WENO5-JS face value (same formula as weno5_face) with one reciprocal:
// alpha_k = d_k / e_k^2 (e_k = eps + indicator k) is multiplied through by
// e_0^2 e_1^2 e_2^2, which cancels between numerator and denominator.  With
// e_k >= eps = 1e-6 every product stays far inside the single-precision range.
template <typename T>
__device__ __forceinline__ T weno5_rcp(T h0, T h1, T h2, T h3, T h4, T a0, T a1, T a2, T a3, T a4,
                                       T eps) {
    const T q0 = ((T)2 * h0 - (T)7 * h1 + (T)11 * h2);
    const T q1 = (-h1 + (T)5 * h2 + (T)2 * h3);
    const T q2 = ((T)2 * h2 + (T)5 * h3 - h4);
    T t = a0 - (T)2 * a1 + a2, s = a0 - (T)4 * a1 + (T)3 * a2;
    const T e0 = eps + ((T)(13.0 / 12.0) * t * t + (T)0.25 * s * s);
    t = a1 - (T)2 * a2 + a3;
    s = a1 - a3;
    const T e1 = eps + ((T)(13.0 / 12.0) * t * t + (T)0.25 * s * s);
    t = a2 - (T)2 * a3 + a4;
    s = (T)3 * a2 - (T)4 * a3 + a4;
    const T e2 = eps + ((T)(13.0 / 12.0) * t * t + (T)0.25 * s * s);
    const T s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    const T b0 = (T)0.1 * (s1 * s2), b1 = (T)0.6 * (s0 * s2), b2 = (T)0.3 * (s0 * s1);
    return (b0 * q0 + b1 * q1 + b2 * q2) * fast_rcp<T>((T)6 * (b0 + b1 + b2));
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
        hh = weno5_rcp<T>(W0 * A0, W1 * A1, W2 * A2, W3 * A3, W4 * A4, A0, A1, A2, A3, A4, eps);
    } else if constexpr (SCHEME == LBW_WENO3) {
        const T A0 = pos ? a1 : a4, A1 = pos ? a2 : a3, A2 = pos ? a3 : a2;
        const T W0 = pos ? w1 : w4, W1 = pos ? w2 : w3, W2 = pos ? w3 : w2;
        hh = weno3_rcp<T>(W0 * A0, W1 * A1, W2 * A2, A0, A1, A2, eps);
    } else {
        hh = pos ? w2 * a2 : w3 * a3;
    }
    return hh - kappa * (a3 - a2);
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

template <typename T, int D, int SCHEME, int STAGE, int TX, int TY>
__device__ __forceinline__ void stage_tile(const RunDev &r, const TileGeom &g, int bx, int by, int bz) {
    constexpr int NT = TX * TY;
    constexpr int AX = TX + 6;                  // a plane row length (x halo 3 + 3)
    constexpr int AY = (D == 3) ? TY + 6 : 1;   // a plane rows
    __shared__ T sA[AY * AX];
    __shared__ T sUx[TY * AX];
    __shared__ T sUy[(D == 3) ? (TY + 6) * TX : 1];
    __shared__ T sFx[TY * (TX + 1)];
    __shared__ T sFy[(D == 3) ? (TY + 1) * TX : 1];

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = bx * TX, y0 = by * TY;
    const int gxl = x0 + tx, gyl = y0 + ty;         // own column (may be outside)
    const bool active = gxl < g.nx && (D == 2 || gyl < g.ny);
    const int xw = active ? gxl : gxl % g.nx;       // wrapped column for loads
    const int yw = (D == 3) ? (active ? gyl : gyl % g.ny) : 0;
    const int64_t col = (int64_t)xw + (int64_t)g.nx * yw;
    const int v0 = bz * g.chunk;
    const int v1 = min(v0 + g.chunk, g.nv);

    const T *__restrict__ C = (const T *)r.c;
    const T *__restrict__ ain = (const T *)(STAGE == 1 ? r.c : (STAGE == 2 ? r.c1 : r.c2));
    const T *__restrict__ ux = (const T *)r.u;
    const T *__restrict__ uy = ux + g.N;
    const T *__restrict__ uv = ux + (int64_t)(D - 1) * g.N;
    const T vs = (T)r.vs, kap = (T)r.kappa_c, eps = (T)r.eps;
    const bool walls = !g.vper;

    // vertical index with the wall/periodic rule; sets flip for mirrored nodes
    auto vidx = [&](int v, bool &flip) -> int {
        flip = false;
        if (!walls) {
            v %= g.nv;
            return v < 0 ? v + g.nv : v;
        }
        if (v < 0) { flip = true; return -1 - v; }
        if (v >= g.nv) { flip = true; return 2 * g.nv - 1 - v; }
        return v;
    };
    auto load_av = [&](int v, T &a, T &w) {
        bool flip;
        const int vv = vidx(v, flip);
        const int64_t k = col + (int64_t)vv * g.sv;
        a = ain[k];
        const T u = uv[k];
        w = (flip ? -u : u) - vs;
    };

    // lateral halo slots of this thread (fixed over the march)
    // a-plane cross: rows ty in [0,TY) x cols [0,AX), plus (3D) y-halo rows
    constexpr int NA = (D == 3) ? AX * TY + TX * 6 : AX;
    constexpr int NUX = AX * TY;
    constexpr int NUY = (D == 3) ? TX * (TY + 6) : 0;
    constexpr int SA = (NA + NT - 1) / NT, SUX = (NUX + NT - 1) / NT, SUY = (NUY + NT - 1) / NT;
    int64_t offA[SA];
    int ldsA[SA];
    int64_t offX[SUX];
    int ldsX[SUX];
    int64_t offY[(SUY > 0) ? SUY : 1];
    int ldsY[(SUY > 0) ? SUY : 1];
    auto wrapx = [&](int x) { x %= g.nx; return x < 0 ? x + g.nx : x; };
    auto wrapy = [&](int y) { y %= g.ny; return y < 0 ? y + g.ny : y; };
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        const int i = tid + s * NT;
        ldsA[s] = -1;
        offA[s] = 0;
        if (i < NA) {
            int lx, ly;  // plane-local coords, halo origin at (-3, -3)
            if (i < AX * TY) { lx = i % AX; ly = (D == 3) ? (i / AX) + 3 : 0; }
            else { const int j = i - AX * TY; lx = (j % TX) + 3; ly = (j / TX) < 3 ? (j / TX) : (j / TX) + TY; }
            const int gxx = wrapx(x0 + lx - 3);
            const int gyy = (D == 3) ? wrapy(y0 + ly - 3) : 0;
            offA[s] = (int64_t)gxx + (int64_t)g.nx * gyy;
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
            const int gxx = wrapx(x0 + lx - 3);
            const int gyy = (D == 3) ? wrapy(y0 + ly) : 0;
            offX[s] = (int64_t)gxx + (int64_t)g.nx * gyy;
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
            const int gxx = wrapx(x0 + lx);
            const int gyy = wrapy(y0 + ly - 3);
            offY[s] = (int64_t)gxx + (int64_t)g.nx * gyy;
            ldsY[s] = ly * TX + lx;
        }
    }

    // vertical windows: a and w at v-2 .. v+3 for the face above v
    T aw[6], ww[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) load_av(v0 - 2 + m, aw[m], ww[m]);
    // face below the first plane
    T fbelow;
    if (walls && v0 == 0) {
        fbelow = -vs * aw[2];                       // absorbing bottom
    } else {
        T ab, wb;
        load_av(v0 - 3, ab, wb);
        fbelow = face6<T, SCHEME>(ab, aw[0], aw[1], aw[2], aw[3], aw[4], wb, ww[0], ww[1], ww[2],
                                  ww[3], ww[4], kap, eps);
    }

    // prefetch registers for the lateral planes
    T pA[SA], pX[SUX], pY[(SUY > 0) ? SUY : 1];
    auto prefetch = [&](int v) {
        bool flip;
        const int vv = vidx(v, flip);
        const int64_t base = (int64_t)vv * g.sv;
#pragma unroll
        for (int s = 0; s < SA; ++s) pA[s] = ldsA[s] >= 0 ? ain[base + offA[s]] : (T)0;
#pragma unroll
        for (int s = 0; s < SUX; ++s) pX[s] = ldsX[s] >= 0 ? ux[base + offX[s]] : (T)0;
#pragma unroll
        for (int s = 0; s < SUY; ++s) pY[s] = ldsY[s] >= 0 ? uy[base + offY[s]] : (T)0;
    };
    prefetch(v0);

    for (int v = v0; v < v1; ++v) {
        // publish plane v
#pragma unroll
        for (int s = 0; s < SA; ++s) if (ldsA[s] >= 0) sA[ldsA[s]] = pA[s];
#pragma unroll
        for (int s = 0; s < SUX; ++s) if (ldsX[s] >= 0) sUx[ldsX[s]] = pX[s];
#pragma unroll
        for (int s = 0; s < SUY; ++s) if (ldsY[s] >= 0) sUy[ldsY[s]] = pY[s];
        __syncthreads();
        // next plane's loads in flight while this one is computed
        if (v + 1 < v1) prefetch(v + 1);
        T anext, wnext;
        load_av(v + 4, anext, wnext);
        const int64_t kc = col + (int64_t)v * g.sv;
        T cown = (T)0;
        if (STAGE != 1) cown = C[kc];

        // lateral faces: x faces (TX+1 per row), then y faces (TY+1 per column)
        for (int i = tid; i < TY * (TX + 1); i += NT) {
            const int fx = i % (TX + 1), fy = i / (TX + 1);  // face between local fx-1 and fx
            const T *ar = sA + ((D == 3) ? (fy + 3) : 0) * AX + fx;   // node fx-3 .. fx+2 -> +0..+5
            const T *ur = sUx + fy * AX + fx;
            sFx[fy * (TX + 1) + fx] = face6<T, SCHEME>(ar[0], ar[1], ar[2], ar[3], ar[4], ar[5], ur[0],
                                                        ur[1], ur[2], ur[3], ur[4], ur[5], kap, eps);
        }
        if constexpr (D == 3) {
            for (int i = tid; i < (TY + 1) * TX; i += NT) {
                const int fx = i % TX, fy = i / TX;   // face between local rows fy-1 and fy
                const T *ac = sA + fy * AX + fx + 3;   // rows fy-3+3 .. : column fx
                const T *uc = sUy + fy * TX + fx;
                sFy[fy * TX + fx] = face6<T, SCHEME>(ac[0], ac[AX], ac[2 * AX], ac[3 * AX], ac[4 * AX],
                                                     ac[5 * AX], uc[0], uc[TX], uc[2 * TX], uc[3 * TX],
                                                     uc[4 * TX], uc[5 * TX], kap, eps);
            }
        }
        // vertical face above this cell
        T fabove;
        if (walls && v == g.nv - 1)
            fabove = (T)0;
        else
            fabove = face6<T, SCHEME>(aw[0], aw[1], aw[2], aw[3], aw[4], aw[5], ww[0], ww[1], ww[2],
                                      ww[3], ww[4], ww[5], kap, eps);
        __syncthreads();
        T L = -(fabove - fbelow);
        L -= sFx[ty * (TX + 1) + tx + 1] - sFx[ty * (TX + 1) + tx];
        if constexpr (D == 3) L -= sFy[(ty + 1) * TX + tx] - sFy[ty * TX + tx];
        const T a = aw[2];
        if (active) {
            if constexpr (STAGE == 1) {
                ((T *)r.c1)[kc] = a + L;
            } else if constexpr (STAGE == 2) {
                ((T *)r.c2)[kc] = (T)0.75 * cown + (T)0.25 * a + (T)0.25 * L;
            } else {
                if (walls && v == 0) {
                    const double o0 = r.vs * (double)cown;
                    const double o1 = r.vs * (double)((const T *)r.c1)[kc];
                    const double o2 = r.vs * (double)a;
                    r.dep[col] += o0 / 6.0 + o1 / 6.0 + 2.0 / 3.0 * o2;
                }
                ((T *)r.c)[kc] = cown / (T)3 + (T)(2.0 / 3.0) * a + (T)(2.0 / 3.0) * L;
            }
        }
        fbelow = fabove;
#pragma unroll
        for (int m = 0; m < 5; ++m) { aw[m] = aw[m + 1]; ww[m] = ww[m + 1]; }
        aw[5] = anext;
        ww[5] = wnext;
        __syncthreads();
    }
}

template <typename T, int D, int SCHEME, int STAGE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_stage_tiled(RunDev r, TileGeom g) {
    int bx, by, bz;
    block_tile(g, bx, by, bz);
    stage_tile<T, D, SCHEME, STAGE, TX, TY>(r, g, bx, by, bz);
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
template <typename T, int D, int SCHEME, int STAGE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_stage_batched(const RunDev *__restrict__ runs,
                                                          const int *__restrict__ tile_start,
                                                          int nbatch, int chunk, int sflip) {
    const int total = tile_start[nbatch];
    const int G = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per_xcd = (G + 7 - xcd) >> 3;               // blocks on this XCD
    const int lo = (int)((int64_t)total * xcd / 8), hi = (int)((int64_t)total * (xcd + 1) / 8);
    for (int w = lo + slot; w < hi; w += per_xcd) {
        int b = 0;
        while (tile_start[b + 1] <= w) ++b;                // runs are few; linear scan
        RunDev r = runs[b];
        if (sflip) { void *t = r.s; r.s = r.s2; r.s2 = t; }
        const TileGeom g = make_geom<D>(r, chunk, TX, TY);
        const int t = w - tile_start[b];
        const int bx = t % g.gx, rest = t / g.gx;
        stage_tile<T, D, SCHEME, STAGE, TX, TY>(r, g, bx, rest % g.gy, rest / g.gy);
    }
}

template <typename T, int D, int SCHEME, int TX, int TY>
hipError_t stages(const RunDev &r, int chunk, hipStream_t st) {
    const TileGeom g = make_geom<D>(r, chunk, TX, TY);
    const int64_t nb = (int64_t)g.gx * g.gy * g.gz;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    k_stage_tiled<T, D, SCHEME, 1, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    k_stage_tiled<T, D, SCHEME, 2, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (r.has_s) {
        e = launch_s_update(D, sizeof(T) == 4 ? LBW_FP32_SHIFTED : LBW_FP64, r, st);
        if (e != hipSuccess) return e;
    }
    k_stage_tiled<T, D, SCHEME, 3, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    return hipGetLastError();
}

template <typename T, int D, int SCHEME, int TX, int TY>
hipError_t stage_slab_t(const RunDev &r, int chunk, int stage, int v_lo, int v_hi, hipStream_t st) {
    TileGeom g = make_geom<D>(r, chunk, TX, TY);
    const int c0 = v_lo / g.chunk, c1 = (v_hi + g.chunk - 1) / g.chunk;
    if (v_lo % g.chunk || c1 > g.gz || c0 >= c1) return hipErrorInvalidValue;
    g.bz0 = c0;
    g.gz = c1 - c0;
    const int64_t nb = (int64_t)g.gx * g.gy * g.gz;
    if (stage == 1) k_stage_tiled<T, D, SCHEME, 1, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    else if (stage == 2) k_stage_tiled<T, D, SCHEME, 2, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    else k_stage_tiled<T, D, SCHEME, 3, TX, TY><<<(unsigned)nb, TX * TY, 0, st>>>(r, g);
    return hipGetLastError();
}

template <typename T, int D, int SCHEME>
hipError_t stage_slab_shape(const RunDev &r, const lbw_launch &l, int stage, int v_lo, int v_hi,
                            hipStream_t st) {
    const TileShape sh = resolve_tile_shape(D, l);
    if constexpr (D == 3) {
        if (sh.tx == 64) return stage_slab_t<T, D, SCHEME, 64, 4>(r, sh.chunk, stage, v_lo, v_hi, st);
        if (sh.tx == 128) return stage_slab_t<T, D, SCHEME, 128, 2>(r, sh.chunk, stage, v_lo, v_hi, st);
        return stage_slab_t<T, D, SCHEME, 32, 8>(r, sh.chunk, stage, v_lo, v_hi, st);
    } else {
        if (sh.tx == 64) return stage_slab_t<T, D, SCHEME, 64, 1>(r, sh.chunk, stage, v_lo, v_hi, st);
        if (sh.tx == 128) return stage_slab_t<T, D, SCHEME, 128, 1>(r, sh.chunk, stage, v_lo, v_hi, st);
        return stage_slab_t<T, D, SCHEME, 256, 1>(r, sh.chunk, stage, v_lo, v_hi, st);
    }
}

template <typename T, int D>
hipError_t stage_slab_d(const RunDev &r, const lbw_launch &l, int stage, int v_lo, int v_hi,
                        hipStream_t st) {
    switch (r.scheme) {
        case LBW_WENO5: return stage_slab_shape<T, D, LBW_WENO5>(r, l, stage, v_lo, v_hi, st);
        case LBW_WENO3: return stage_slab_shape<T, D, LBW_WENO3>(r, l, stage, v_lo, v_hi, st);
        case LBW_UPWIND1: return stage_slab_shape<T, D, LBW_UPWIND1>(r, l, stage, v_lo, v_hi, st);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D, int SCHEME, int TX, int TY>
hipError_t stages_batched(const BatchArgs &a, hipStream_t st) {
    k_stage_batched<T, D, SCHEME, 1, TX, TY><<<a.grid, TX * TY, 0, st>>>(a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip);
    k_stage_batched<T, D, SCHEME, 2, TX, TY><<<a.grid, TX * TY, 0, st>>>(a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.host_runs[0].has_s) {
        for (int b = 0; b < a.nbatch; ++b) {
            RunDev r = a.host_runs[b];
            if (a.sflip) { void *t = r.s; r.s = r.s2; r.s2 = t; }
            e = launch_s_update(D, sizeof(T) == 4 ? LBW_FP32_SHIFTED : LBW_FP64, r, st);
            if (e != hipSuccess) return e;
        }
    }
    k_stage_batched<T, D, SCHEME, 3, TX, TY><<<a.grid, TX * TY, 0, st>>>(a.runs, a.tile_start, a.nbatch, a.chunk, a.sflip);
    return hipGetLastError();
}

template <typename T, int D, int SCHEME>
hipError_t stages_shape(const RunDev &r, const lbw_launch &l, hipStream_t st, const BatchArgs *batch) {
    const TileShape sh = resolve_tile_shape(D, l);
    if (batch) {
        if constexpr (D == 3) {
            if (sh.tx == 64) return stages_batched<T, D, SCHEME, 64, 4>(*batch, st);
            if (sh.tx == 128) return stages_batched<T, D, SCHEME, 128, 2>(*batch, st);
            return stages_batched<T, D, SCHEME, 32, 8>(*batch, st);
        } else {
            if (sh.tx == 64) return stages_batched<T, D, SCHEME, 64, 1>(*batch, st);
            if (sh.tx == 128) return stages_batched<T, D, SCHEME, 128, 1>(*batch, st);
            return stages_batched<T, D, SCHEME, 256, 1>(*batch, st);
        }
    }
    if constexpr (D == 3) {
        if (sh.tx == 64) return stages<T, D, SCHEME, 64, 4>(r, sh.chunk, st);
        if (sh.tx == 128) return stages<T, D, SCHEME, 128, 2>(r, sh.chunk, st);
        return stages<T, D, SCHEME, 32, 8>(r, sh.chunk, st);
    } else {
        if (sh.tx == 64) return stages<T, D, SCHEME, 64, 1>(r, sh.chunk, st);
        if (sh.tx == 128) return stages<T, D, SCHEME, 128, 1>(r, sh.chunk, st);
        return stages<T, D, SCHEME, 256, 1>(r, sh.chunk, st);
    }
}

template <typename T, int D>
hipError_t tiled_d(const RunDev &r, const lbw_launch &l, hipStream_t st, const BatchArgs *b) {
    switch (r.scheme) {
        case LBW_WENO5: return stages_shape<T, D, LBW_WENO5>(r, l, st, b);
        case LBW_WENO3: return stages_shape<T, D, LBW_WENO3>(r, l, st, b);
        case LBW_UPWIND1: return stages_shape<T, D, LBW_UPWIND1>(r, l, st, b);
    }
    return hipErrorInvalidValue;
}

}  // namespace

TileShape resolve_tile_shape(int dim, const lbw_launch &l) {
    TileShape s;
    if (dim == 3) {
        s.tx = (l.tile_x == 64 || l.tile_x == 128) ? l.tile_x : 32;
        s.ty = 256 / s.tx;
    } else {
        s.tx = (l.tile_x == 64 || l.tile_x == 128) ? l.tile_x : 256;
        s.ty = 1;
    }
    s.chunk = l.tile_y > 0 ? l.tile_y : (dim == 3 ? 64 : 32);
    return s;
}

int64_t transport_tiles(int dim, const RunDev &r, const lbw_launch &l) {
    const TileShape s = resolve_tile_shape(dim, l);
    const TileGeom g = dim == 3 ? make_geom<3>(r, s.chunk, s.tx, s.ty) : make_geom<2>(r, s.chunk, s.tx, s.ty);
    return (int64_t)g.gx * g.gy * g.gz;
}

hipError_t launch_transport_tiled(int dim, int precision, const RunDev &r, const lbw_launch &l,
                                  hipStream_t st) {
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? tiled_d<float, 2>(r, l, st, nullptr) : tiled_d<float, 3>(r, l, st, nullptr);
    return dim == 2 ? tiled_d<double, 2>(r, l, st, nullptr) : tiled_d<double, 3>(r, l, st, nullptr);
}

hipError_t launch_stage_slab(int dim, int precision, const RunDev &r, const lbw_launch &l,
                             int stage, int v_lo, int v_hi, hipStream_t st) {
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? stage_slab_d<float, 2>(r, l, stage, v_lo, v_hi, st)
                        : stage_slab_d<float, 3>(r, l, stage, v_lo, v_hi, st);
    return dim == 2 ? stage_slab_d<double, 2>(r, l, stage, v_lo, v_hi, st)
                    : stage_slab_d<double, 3>(r, l, stage, v_lo, v_hi, st);
}

hipError_t launch_transport_batched(int dim, int precision, const BatchArgs &b, const lbw_launch &l,
                                    hipStream_t st) {
    const RunDev &r = b.host_runs[0];
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? tiled_d<float, 2>(r, l, st, &b) : tiled_d<float, 3>(r, l, st, &b);
    return dim == 2 ? tiled_d<double, 2>(r, l, st, &b) : tiled_d<double, 3>(r, l, st, &b);
}

}  // namespace lbw
