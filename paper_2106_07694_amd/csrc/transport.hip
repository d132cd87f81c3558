// transport.hip -- scalar transport part of the coupled step (supplement
// section 1): the particle concentration C advances by the TVD-RK3 scheme of
// S21-S23 with the transport velocity w = u - Vs e_v frozen at time level n,
//
//   a1 = C + L(C),  a2 = 3/4 C + 1/4 a1 + 1/4 L(a1),  C+ = 1/3 C + 2/3 a2 + 2/3 L(a2),
//
// where L(a) = -sum over axes of the face-flux differences (conservative form
// of eq. 6).  Faces on the lateral axes wrap periodically.  On the vertical
// axis with walls, stencils that reach past a wall see the mirror image of the
// field (zero normal gradient, eq. 14-15) and of the fluid's vertical velocity
// with its sign flipped (no penetration), settling unchanged; the top wall
// face carries no flux and the bottom wall face carries the settling flux
// -Vs a_0 out of the domain into the per-column deposit counter, weighted
// 1/6, 1/6, 2/3 over the three stages so that sum C + deposit is conserved.
// S (when present) takes one forward-Euler step of first-order upwind in
// conservative form (S5-S6) with central diffusion and closed walls.
//
// This unit holds the plain global-memory kernels: one thread per node,
// stencil values read through the caches.
#include "transport_device.h"

namespace lbw {
namespace {

template <int D>
__device__ __forceinline__ void node_coords(const RunDev &r, int64_t k, int &x, int &y, int &z) {
    x = (int)(k % r.nx);
    const int64_t t = k / r.nx;
    if constexpr (D == 2) {
        y = (int)t;
        z = 0;
    } else {
        y = (int)(t % r.ny);
        z = (int)(t / r.ny);
    }
}

// Settling speed of C at node k: vs, or Vs (1 - vs_s S_k) when the speed is
// set by the local fluid density (eq. 13 with rho linear in S).
template <typename T>
__device__ __forceinline__ T settling_at(const RunDev &r, T vs, int64_t k) {
    if (r.vs_s == 0.0) return vs;
    return vs * ((T)1 - (T)r.vs_s * ((const T *)r.s)[k]);
}

// L(a) at node k.  absorbing: bottom wall face carries -Vs*a_0 (C, with the
// settling speed of settling_at); otherwise the walls are closed and nothing
// settles (S).
template <typename T, int D, int SCHEME, bool ABSORB>
__device__ T spatial_op(const RunDev &r, const T *__restrict__ a, const T *__restrict__ u,
                        int64_t k, int x, int y, int z, T vs, T kappa, T eps) {
    T L = 0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        const bool vert = (ax == D - 1);
        const bool walls = vert && !r.vper;
        const int j = ax == 0 ? x : (ax == 1 ? y : z);
        const int n = ax == 0 ? r.nx : (ax == 1 ? r.ny : r.nz);
        const int64_t stride = ax == 0 ? 1 : (ax == 1 ? (int64_t)r.nx : (int64_t)r.nx * r.ny);
        T av[7], wv[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            int jj = j + m - 3;
            bool ghost = false;
            if (!walls) {
                jj = ((jj % n) + n) % n;
            } else if (jj < 0) {
                jj = -1 - jj;
                ghost = true;
            } else if (jj >= n) {
                jj = 2 * n - 1 - jj;
                ghost = true;
            }
            const int64_t kk = k + (int64_t)(jj - j) * stride;
            av[m] = a[kk];
            T uu = u[(int64_t)ax * r.N + kk];
            if (ghost) uu = -uu;
            wv[m] = vert ? uu - (ABSORB ? settling_at<T>(r, vs, kk) : vs) : uu;
        }
        const T Fp = (walls && j == n - 1) ? (T)0 : face_flux<T, SCHEME>(av + 1, wv + 1, kappa, eps);
        const T Fm = (walls && j == 0) ? (ABSORB ? -settling_at<T>(r, vs, k) * av[3] : (T)0)
                                       : face_flux<T, SCHEME>(av, wv, kappa, eps);
        L -= (Fp - Fm);
    }
    return L;
}

template <typename T, int D, int SCHEME, int STAGE>
__global__ void __launch_bounds__(256) k_rk_stage(RunDev r) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    node_coords<D>(r, k, x, y, z);
    T *__restrict__ C = (T *)r.c;
    const T *__restrict__ ain = (const T *)(STAGE == 1 ? r.c : (STAGE == 2 ? r.c1 : r.c2));
    const T *__restrict__ u = (const T *)r.u;
    const T vs = (T)r.vs;
    const T L = spatial_op<T, D, SCHEME, true>(r, ain, u, k, x, y, z, vs, (T)r.kappa_c, (T)r.eps);
    const T a = ain[k];
    if constexpr (STAGE == 1) {
        ((T *)r.c1)[k] = a + L;
    } else if constexpr (STAGE == 2) {
        ((T *)r.c2)[k] = rk3_stage2<T>(C[k], a, L);
    } else {
        const T c0 = C[k];
        const int v = (D == 2) ? y : z;
        if (!r.vper && v == 0) {
            // settled mass through the bottom face over the three stages
            const double vsd = r.vs * (1.0 - r.vs_s * (r.vs_s == 0.0 ? 0.0 : (double)((const T *)r.s)[k]));
            const double o0 = vsd * (double)c0;
            const double o1 = vsd * (double)((const T *)r.c1)[k];
            const double o2 = vsd * (double)a;
            const int64_t col = (D == 2) ? x : (int64_t)x + (int64_t)r.nx * y;
            r.dep[col] += o0 / 6.0 + o1 / 6.0 + 2.0 / 3.0 * o2;
        }
        C[k] = rk3_stage3<T>(c0, a, L);
    }
}

// S update (S5-S6 in conservative form, R13): forward Euler of the
// first-order upwind flux of h = u S plus central diffusion, closed walls,
// nothing settles.  One thread per node of a plane, the planes of [v_lo,
// v_hi) across grid.y (strided when there are more than grid.y of them);
// coordinates are 32-bit within a plane (a plane holds fewer than 2^29
// cells, checked at creation) and only the neighbours the first-order flux
// reads are loaded.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_s_update(RunDev r, int v_lo, int v_hi) {
    const int nx = r.nx, ny = (D == 3) ? r.ny : 1, nv = (D == 3) ? r.nz : r.ny;
    const int P = nx * ny;
    const int p = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (p >= P) return;
    const int x = p % nx, y = (D == 3) ? p / nx : 0;
    const T *__restrict__ s = (const T *)r.s;
    const T *__restrict__ ux = (const T *)r.u;
    const T *__restrict__ uy = ux + r.N;
    const T *__restrict__ uv = ux + (int64_t)(D - 1) * r.N;
    const T kap = (T)r.kappa_s;
    // face between nodes j (a2, w2) and j + 1 (a3, w3)
    auto face = [&](T a2, T a3, T w2, T w3) -> T {
        const T hh = ((T)0.5 * (w2 + w3) >= (T)0) ? w2 * a2 : w3 * a3;
        return hh - kap * (a3 - a2);
    };
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    for (int v = v_lo + (int)blockIdx.y; v < v_hi; v += (int)gridDim.y) {
        const int64_t k = (int64_t)v * P + p;
        const T s0 = s[k];
        const int64_t kxm = k + (xm - x), kxp = k + (xp - x);
        T L = -(face(s0, s[kxp], ux[k], ux[kxp]) - face(s[kxm], s0, ux[kxm], ux[k]));
        if constexpr (D == 3) {
            const int64_t kym = k + (int64_t)(ym - y) * nx, kyp = k + (int64_t)(yp - y) * nx;
            L -= face(s0, s[kyp], uy[k], uy[kyp]) - face(s[kym], s0, uy[kym], uy[k]);
        }
        const bool top = !r.vper && v == nv - 1, bottom = !r.vper && v == 0;
        const int vm = v == 0 ? nv - 1 : v - 1, vp = v == nv - 1 ? 0 : v + 1;
        const int64_t kvm = k + (int64_t)(vm - v) * P, kvp = k + (int64_t)(vp - v) * P;
        const T Fp = top ? (T)0 : face(s0, s[kvp], uv[k], uv[kvp]);
        const T Fm = bottom ? (T)0 : face(s[kvm], s0, uv[kvm], uv[k]);
        L -= Fp - Fm;
        ((T *)r.s2)[k] = s0 + L;
    }
}

template <typename T, int D, int SCHEME>
hipError_t transport_t(const RunDev &r, hipStream_t st) {
    const int block = 256;
    const dim3 grid((unsigned)((r.N + block - 1) / block));
    k_rk_stage<T, D, SCHEME, 1><<<grid, block, 0, st>>>(r);
    k_rk_stage<T, D, SCHEME, 2><<<grid, block, 0, st>>>(r);
    if (r.has_s) {
        const hipError_t e = launch_s_update(D, sizeof(T) == 4 ? LBW_FP32_SHIFTED : LBW_FP64, r, st);
        if (e != hipSuccess) return e;
    }
    k_rk_stage<T, D, SCHEME, 3><<<grid, block, 0, st>>>(r);
    return hipGetLastError();
}

template <typename T, int D>
hipError_t transport_d(const RunDev &r, hipStream_t st) {
    switch (r.scheme) {
        case LBW_WENO5: return transport_t<T, D, LBW_WENO5>(r, st);
        case LBW_WENO3: return transport_t<T, D, LBW_WENO3>(r, st);
        case LBW_UPWIND1: return transport_t<T, D, LBW_UPWIND1>(r, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_s_update(int dim, int precision, const RunDev &r, hipStream_t st) {
    const int64_t P = (int64_t)r.nx * (dim == 3 ? r.ny : 1);
    const int v_lo = 0, v_hi = dim == 3 ? r.nz : r.ny;
    const dim3 grid((unsigned)((P + 255) / 256), (unsigned)std::min(v_hi - v_lo, 65535));
    if (precision == LBW_FP32_SHIFTED) {
        if (dim == 2) k_s_update<float, 2><<<grid, 256, 0, st>>>(r, v_lo, v_hi);
        else k_s_update<float, 3><<<grid, 256, 0, st>>>(r, v_lo, v_hi);
    } else {
        if (dim == 2) k_s_update<double, 2><<<grid, 256, 0, st>>>(r, v_lo, v_hi);
        else k_s_update<double, 3><<<grid, 256, 0, st>>>(r, v_lo, v_hi);
    }
    return hipGetLastError();
}

hipError_t launch_transport(int dim, int precision, const RunDev &r, const lbw_launch &l,
                            hipStream_t st) {
    if (l.variant != 1) return launch_transport_tiled(dim, precision, r, l, st);
    if (precision == LBW_FP32_SHIFTED)
        return dim == 2 ? transport_d<float, 2>(r, st) : transport_d<float, 3>(r, st);
    return dim == 2 ? transport_d<double, 2>(r, st) : transport_d<double, 3>(r, st);
}

}  // namespace lbw
