// lbm_device.h -- device helpers of the in-place streaming scheme shared by
// the collide-stream, export, reduction and adjoint kernels.
#pragma once

#include "lbw_internal.h"

namespace lbw {

// Linear index of the node displaced by (dx, dy, dz) from (x, y, z): lateral
// axes wrap; on the vertical axis with walls the result is -1 below the
// bottom wall and -2 above the top wall.
template <int D>
__device__ __forceinline__ int64_t displaced(const RunDev &r, int x, int y, int z, int dx,
                                             int dy, int dz) {
    int xs = x + dx;
    xs += (xs < 0) ? r.nx : 0;
    xs -= (xs >= r.nx) ? r.nx : 0;
    if constexpr (D == 2) {
        int ys = y + dy;
        if (r.vper) {
            ys += (ys < 0) ? r.ny : 0;
            ys -= (ys >= r.ny) ? r.ny : 0;
        } else {
            if (ys < 0) return -1;
            if (ys >= r.ny) return -2;
        }
        return (int64_t)xs + (int64_t)r.nx * ys;
    } else {
        int ys = y + dy;
        ys += (ys < 0) ? r.ny : 0;
        ys -= (ys >= r.ny) ? r.ny : 0;
        int zs = z + dz;
        if (r.vper) {
            zs += (zs < 0) ? r.nz : 0;
            zs -= (zs >= r.nz) ? r.nz : 0;
        } else {
            if (zs < 0) return -1;
            if (zs >= r.nz) return -2;
        }
        return (int64_t)xs + (int64_t)r.nx * ((int64_t)ys + (int64_t)r.ny * zs);
    }
}

// Population accesses of the collide-stream kernels: NT marks them
// non-temporal (streamed past the caches), which pays when the populations
// are far larger than the last-level cache and costs when they fit in it.
template <typename T, bool NT>
__device__ __forceinline__ T pop_load(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename T, bool NT>
__device__ __forceinline__ void pop_store(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// 6 w_i (c_i . u_top): momentum a moving top wall hands to a reflected
// population (half-way bounce-back with a wall velocity).
// The components with c_i = 0 are left out of the sum (each kept product is
// exact, c_i being +-1), so for an unrolled i only the wall's tangential
// and normal parts that the direction carries are computed.
template <int Q>
__device__ __forceinline__ double lid_term(const RunDev &r, int i) {
    using L = Lattice<Q>;
    double cu = 0.0;
    if (L::cx[i]) cu = L::cx[i] * r.utop[0];
    if (L::cy[i]) cu = cu + L::cy[i] * r.utop[1];
    if (L::cz[i]) cu = cu + L::cz[i] * r.utop[2];
    return 6.0 * L::w[i] * cu;
}

// Canonical pre-collision population f_i at node k when the buffer holds the
// state after an even-step kernel (odd = true) or after an odd-step kernel.
template <int Q, typename T, bool NT = false>
__device__ __forceinline__ T load_canonical(const RunDev &r, const T *__restrict__ f, int i,
                                            int64_t k, int x, int y, int z, bool odd) {
    using L = Lattice<Q>;
    if (!odd) return pop_load<T, NT>(&f[(int64_t)i * r.N + k]);
    const int64_t src = displaced<L::D>(r, x, y, z, -L::cx[i], -L::cy[i], -L::cz[i]);
    if (src >= 0) return pop_load<T, NT>(&f[(int64_t)L::opp[i] * r.N + src]);
    T v = pop_load<T, NT>(&f[(int64_t)i * r.N + k]);
    if (src == -2) v += (T)lid_term<Q>(r, i);  // f_i = f*_opp(i) + 6 w_i c_i.u_top
    return v;
}

template <int D>
__device__ __forceinline__ void coords(const RunDev &r, int64_t k, int &x, int &y, int &z) {
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

// Inverse of load_canonical: place the canonical value v of f_i at node k
// where the next kernel of the pair expects it.
template <int Q, typename T>
__device__ __forceinline__ void store_canonical(const RunDev &r, T *__restrict__ f, int i,
                                                int64_t k, int x, int y, int z, bool odd, T v) {
    using L = Lattice<Q>;
    if (!odd) {
        f[(int64_t)i * r.N + k] = v;
        return;
    }
    const int64_t src = displaced<L::D>(r, x, y, z, -L::cx[i], -L::cy[i], -L::cz[i]);
    if (src >= 0) {
        f[(int64_t)L::opp[i] * r.N + src] = v;
    } else {
        if (src == -2) v -= (T)lid_term<Q>(r, i);
        f[(int64_t)i * r.N + k] = v;
    }
}

// Density and force-shifted velocity of one node's populations (eq. 19-20
// with rho u = sum f c + F/2, eq. 22); shifted storage holds f_i - w_i.  The
// forward step and its adjoint both use this, so they agree bit for bit.
template <int Q, typename T, bool SH>
__device__ __forceinline__ void lbm_rho_u(const T (&fi)[Q], const T F[3], T &rho, T &drho,
                                          T u[3]) {
#pragma clang fp contract(on)
    using L = Lattice<Q>;
    T r = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r += fi[i];
        if (L::cx[i]) mx += L::cx[i] > 0 ? fi[i] : -fi[i];
        if (L::cy[i]) my += L::cy[i] > 0 ? fi[i] : -fi[i];
        if (L::D == 3 && L::cz[i]) mz += L::cz[i] > 0 ? fi[i] : -fi[i];
    }
    drho = SH ? r : r - (T)1;
    rho = SH ? (T)1 + r : r;
    const T inv = (T)1 / rho;
    u[0] = (mx + (T)0.5 * F[0]) * inv;
    u[1] = (my + (T)0.5 * F[1]) * inv;
    u[2] = (L::D == 3) ? (mz + (T)0.5 * F[2]) * inv : (T)0;
}

// Force density at node k: body force plus the buoyancy of C and S on the
// vertical axis (eq. 10, linear in C and S), -gp_c C - gp_s S (1 - phi_c C):
// the density anomaly of the fluid acts on its fraction 1 - phi, phi =
// phi_c C (phi_c = 0: the linear form).  With several particle size classes
// C is their total, summed in class order (eq. 11-12).
// The same from the total concentration ctot and S (sv, read only with S).
template <int D, typename T>
__device__ __forceinline__ void lbm_force_of(const RunDev &r, T ctot, T sv, T F[3]) {
#pragma clang fp contract(on)
    T fv = -(T)r.gp_c * ctot;
    if (r.has_s) fv -= (T)r.gp_s * (sv * ((T)1 - (T)r.phi_c * ctot));
    F[0] = (T)r.body[0];
    F[1] = (T)r.body[1] + (D == 2 ? fv : (T)0);
    F[2] = (T)r.body[2] + (D == 3 ? fv : (T)0);
}

template <int D, typename T>
__device__ __forceinline__ void lbm_force(const RunDev &r, const T *__restrict__ c,
                                          const T *__restrict__ s, int64_t k, T F[3]) {
    T ctot = c[k];
    for (int i = 1; i < r.ncls; ++i) ctot += c[k + (int64_t)i * r.N];
    lbm_force_of<D, T>(r, ctot, r.has_s ? s[k] : (T)0, F);
}

// c_i . a for the unrolled direction i: the components with c = 0 are left
// out (0 * a is not folded away in IEEE arithmetic, so writing them costs a
// multiply or fused multiply-add each); with c = +-1 every kept product is
// exact, and the sum equals the full one up to the sign of a zero.
template <int Q, typename T>
__device__ __forceinline__ T cdot(int i, T ax, T ay, T az) {
    using L = Lattice<Q>;
    T s = (T)0;
    bool any = false;
    if (L::cx[i]) { s = L::cx[i] > 0 ? ax : -ax; any = true; }
    if (L::cy[i]) { const T t = L::cy[i] > 0 ? ay : -ay; s = any ? s + t : t; any = true; }
    if (L::D == 3 && L::cz[i]) { const T t = L::cz[i] > 0 ? az : -az; s = any ? s + t : t; }
    return s;
}

// BGK collision with Guo forcing (eq. 18, 22) of one node's populations fi
// (in place) for force F, after the moments of eq. 19-20: rho and the
// force-shifted velocity u come back for the caller to store.
//
// Multiply-adds are fused only within one source expression (contract(on)):
// with the default fast contraction the compiler may also fuse across
// statements, differently in each kernel this is inlined into, and the
// in-place pair, its row-staged odd form and the batched form must give the
// same bits.
template <int Q, typename T, bool SH>
__device__ __forceinline__ void lbm_collide(const RunDev &r, T (&fi)[Q], const T F[3], T &rho,
                                            T uu[3]) {
#pragma clang fp contract(on)
    using L = Lattice<Q>;
    T drho;
    lbm_rho_u<Q, T, SH>(fi, F, rho, drho, uu);
    const T Fx = F[0], Fy = F[1], Fz = F[2];
    const T ux = uu[0], uy = uu[1], uz = uu[2];
    const T omega = (T)r.omega, guo = (T)r.guo;
    const T usq = ux * ux + uy * uy + uz * uz;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T w = (T)L::w[i];
        const T cu = cdot<Q>(i, ux, uy, uz);
        const T cF = cdot<Q>(i, Fx, Fy, Fz);
        const T poly = (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * usq;
        // shifted: g_eq = w (drho + rho poly); plain: f_eq = w rho (1 + poly)
        const T feq = SH ? w * (drho + rho * poly) : w * rho * ((T)1 + poly);
        const T Fi = guo * w * ((T)3 * (cF - uF) + (T)9 * cu * cF);
        fi[i] = fi[i] - omega * (fi[i] - feq) + Fi;
    }
}

// Canonical density at node k (shifted storage adds back rho0 = 1).
template <int Q, typename T>
__device__ __forceinline__ T node_density(const RunDev &r, const T *__restrict__ f, int64_t k,
                                          bool odd, bool shifted) {
    using L = Lattice<Q>;
    int x, y, z;
    coords<L::D>(r, k, x, y, z);
    T s = shifted ? (T)1 : (T)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += load_canonical<Q, T>(r, f, i, k, x, y, z, odd);
    return s;
}

}  // namespace lbw
