// adjoint.hip -- reverse mode of one coupled step (WENO5 transport, no S).
//
// Objective sensitivities flow backwards through the step of lbm.hip and
// transport.hip:  J depends on the state at n+1 through (fbar_next of the
// populations, cbar_next of C, dep_bar of every deposit counter); this step
// returns the adjoints of the state at n (fbar, cbar) and adds dJ/dVs.
//
//  1. recompute, from the saved forward state at n: the node velocity u^n
//     (moments, eq. 19-20 with the Guo shift) and the RK stages a1, a2;
//  2. RK3 in reverse (S21-S23 transposed) with the deposit update: each stage
//     needs lam^T dL/da and lam^T dL/du at its input.  The transpose of L is
//     taken face by face: one kernel evaluates every interior face once,
//     multiplies its local Jacobian (six stencil values of a and of the
//     transport velocity, the WENO5 weights differentiated through the
//     smoothness indicators, the upwind side held at its forward choice) by
//     the face's adjoint lam_{j+1} - lam_j and stores the twelve products;
//     a second kernel gathers, for every node, the products of every face
//     stencil that reads it, including stencils that read it as a mirror
//     image beyond a wall (where the vertical velocity enters with a sign
//     flip and the settling speed unchanged);
//  3. streaming in reverse (each population pulls the adjoint from where the
//     forward step sent it), then BGK + Guo collision and the moments in
//     reverse, adding the transport's velocity sensitivity; the force's C
//     dependence closes the loop into cbar.  This runs in the gather kernel
//     of the last reversed stage, once the node's velocity adjoint is whole.
// Every node's adjoint is written by exactly one thread; dJ/dVs is gathered
// per node and summed in a fixed order (FP64).
#include "lbm_device.h"
#include "transport_device.h"

namespace lbw {
namespace {

struct AdjDev {
    RunDev r;
    const void *f_n, *c_n, *rho_n, *fbar_next, *cbar_next;
    void *fbar, *cbar;
    void *u, *a1, *a2, *abar1, *abar2, *ubar, *faceA, *faceW;
    double *vs_part, *partials, *vs_bar;
    double dep_bar;
    int frozen;
    int have_u, have_rho, have_stages;   // forward intermediates supplied by the caller
};

// Periodic index of a position at most three cells outside [0, n): one
// conditional add when n >= 4, the general remainder for tiny axes.
__device__ __forceinline__ int wrap_near(int j, int n) {
    if (n >= 4) return j < 0 ? j + n : (j >= n ? j - n : j);
    j %= n;
    return j < 0 ? j + n : j;
}

template <int D>
__device__ __forceinline__ void xyz(const RunDev &r, int64_t k, int &x, int &y, int &z) {
    coords<D>(r, k, x, y, z);
}

// ---------------------------------------------------------------------------
// 1. moments of the saved populations: u^n (force-shifted)
// ---------------------------------------------------------------------------
template <int Q, typename T, bool SH>
__global__ void __launch_bounds__(256) k_adj_moments(AdjDev a) {
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const RunDev &r = a.r;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    const T *f = (const T *)a.f_n;
    T fi[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) fi[i] = f[(int64_t)i * r.N + k];
    T F[3], u[3], rho, drho;
    lbm_force<D, T>(r, (const T *)a.c_n, nullptr, k, F);
    lbm_rho_u<Q, T, SH>(fi, F, rho, drho, u);
    T *uo = (T *)a.u;
#pragma unroll
    for (int d = 0; d < D; ++d) uo[(int64_t)d * r.N + k] = u[d];
}

// ---------------------------------------------------------------------------
// 2. transpose of the spatial operator
// ---------------------------------------------------------------------------

// Reciprocal: exact in double; the hardware reciprocal (about 1 ulp) in
// single precision.
template <typename T> __device__ __forceinline__ T rcp(T x) { return (T)1 / x; }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Reverse of the WENO5-JS face value for stencil values (upwind -> downwind)
// h (fluxes) and a (smoothness input): gb = dJ/d(face value); returns dJ/dh
// and the smoothness part of dJ/da.  Four reciprocals, no divisions.
template <typename T>
__device__ __forceinline__ void weno5_vjp(const T h[5], const T a[5], T eps, T gb, T hb[5], T ab[5]) {
    constexpr T i6 = (T)(1.0 / 6.0);
    const T q0 = ((T)2 * h[0] - (T)7 * h[1] + (T)11 * h[2]) * i6;
    const T q1 = (-h[1] + (T)5 * h[2] + (T)2 * h[3]) * i6;
    const T q2 = ((T)2 * h[2] + (T)5 * h[3] - h[4]) * i6;
    const T t0 = a[0] - (T)2 * a[1] + a[2], s0 = a[0] - (T)4 * a[1] + (T)3 * a[2];
    const T t1 = a[1] - (T)2 * a[2] + a[3], s1 = a[1] - a[3];
    const T t2 = a[2] - (T)2 * a[3] + a[4], s2 = (T)3 * a[2] - (T)4 * a[3] + a[4];
    const T e0 = eps + ((T)(13.0 / 12.0) * t0 * t0 + (T)0.25 * s0 * s0);
    const T e1 = eps + ((T)(13.0 / 12.0) * t1 * t1 + (T)0.25 * s1 * s1);
    const T e2 = eps + ((T)(13.0 / 12.0) * t2 * t2 + (T)0.25 * s2 * s2);
    const T ie0 = rcp<T>(e0), ie1 = rcp<T>(e1), ie2 = rcp<T>(e2);
    const T al0 = (T)0.1 * ie0 * ie0, al1 = (T)0.6 * ie1 * ie1, al2 = (T)0.3 * ie2 * ie2;
    const T iS = rcp<T>(al0 + al1 + al2);
    const T g = (al0 * q0 + al1 * q1 + al2 * q2) * iS;
    // g = sum al_k q_k / S: dg/dq_k = al_k / S, dg/dal_k = (q_k - g) / S,
    // dal_k/de_k = -2 al_k / e_k (e_k = eps + smoothness indicator k)
    const T gS = gb * iS;
    const T qb0 = gS * al0, qb1 = gS * al1, qb2 = gS * al2;
    const T bb0 = (q0 - g) * qb0 * ((T)-2 * ie0);
    const T bb1 = (q1 - g) * qb1 * ((T)-2 * ie1);
    const T bb2 = (q2 - g) * qb2 * ((T)-2 * ie2);
    hb[0] = (T)(2.0 / 6.0) * qb0;
    hb[1] = (T)(-7.0 / 6.0) * qb0 - i6 * qb1;
    hb[2] = (T)(11.0 / 6.0) * qb0 + (T)(5.0 / 6.0) * qb1 + (T)(2.0 / 6.0) * qb2;
    hb[3] = (T)(2.0 / 6.0) * qb1 + (T)(5.0 / 6.0) * qb2;
    hb[4] = -i6 * qb2;
    // indicator = 13/12 t^2 + 1/4 s^2
    T tb = (T)(13.0 / 6.0) * t0 * bb0, sb = (T)0.5 * s0 * bb0;
    ab[0] = tb + sb;
    ab[1] = (T)-2 * tb - (T)4 * sb;
    ab[2] = tb + (T)3 * sb;
    tb = (T)(13.0 / 6.0) * t1 * bb1;
    sb = (T)0.5 * s1 * bb1;
    ab[1] += tb + sb;
    ab[2] += (T)-2 * tb;
    ab[3] = tb - sb;
    tb = (T)(13.0 / 6.0) * t2 * bb2;
    sb = (T)0.5 * s2 * bb2;
    ab[2] += tb + (T)3 * sb;
    ab[3] += (T)-2 * tb - (T)4 * sb;
    ab[4] = tb + sb;
}

// Products of one face's local Jacobian with its adjoint pb, for the six
// stencil nodes j-2..j+3 (values av, transport velocities wv):
//   A[s] = pb * dPhi/da_s (WENO5 through h = w a and the indicators, plus the
//          central diffusion), W[s] = pb * dPhi/dw_s.
// The upwind side is taken with selects (the stencil is read mirrored when
// the face velocity is negative), so lanes of a wave do not diverge.
template <typename T>
__device__ __forceinline__ void face_vjp(const T av[6], const T wv[6], T pb, T kap, T eps, T A[6],
                                         T W[6]) {
    const bool pos = (wv[2] + wv[3]) >= (T)0;
    T h5[5], a5[5], hb5[5], ab5[5];
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const T aa = pos ? av[s] : av[5 - s];
        const T ww = pos ? wv[s] : wv[5 - s];
        a5[s] = aa;
        h5[s] = ww * aa;
    }
    weno5_vjp<T>(h5, a5, eps, pb, hb5, ab5);
    T hb[6], ab[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const T hp = s < 5 ? hb5[s] : (T)0, hn = s > 0 ? hb5[5 - s] : (T)0;
        const T ap = s < 5 ? ab5[s] : (T)0, an = s > 0 ? ab5[5 - s] : (T)0;
        hb[s] = pos ? hp : hn;
        ab[s] = pos ? ap : an;
    }
    ab[3] += -kap * pb;   // diffusion -kappa (a_{j+1} - a_j)
    ab[2] += kap * pb;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        A[s] = ab[s] + hb[s] * wv[s];   // through a directly and through h = w a
        W[s] = hb[s] * av[s];
    }
}

// For every interior face j+1/2 (stored at its lower node j) and axis d:
//   faceA[d][s] = phibar * dPhi/da_{j-2+s},  faceW[d][s] = phibar * dPhi/dw_{j-2+s}
// with phibar = scale * (lam_{j+1} - lam_j).  Wall faces store zeros.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_adj_face(AdjDev A, const T *__restrict__ a,
                                                  const T *__restrict__ lam, T scale) {
    const RunDev &r = A.r;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    xyz<D>(r, k, x, y, z);
    const T *u = (const T *)(A.frozen ? r.u : A.u);
    T *fa = (T *)A.faceA, *fw = (T *)A.faceW;
    const T vs = (T)r.vs, kap = (T)r.kappa_c, eps = (T)r.eps;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const bool vert = (d == D - 1);
        const bool walls = vert && !r.vper;
        const int j = d == 0 ? x : (d == 1 ? y : z);
        const int n = d == 0 ? r.nx : (d == 1 ? r.ny : r.nz);
        const int64_t stride = d == 0 ? 1 : (d == 1 ? (int64_t)r.nx : (int64_t)r.nx * r.ny);
        const int64_t base = ((int64_t)d * 6) * r.N + k;
        if (walls && j == n - 1) {
#pragma unroll
            for (int s = 0; s < 6; ++s) { fa[base + s * r.N] = (T)0; fw[base + s * r.N] = (T)0; }
            continue;
        }
        T av[6], wv[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            int jj = j + s - 2;
            bool ghost = false;
            if (!walls) jj = wrap_near(jj, n);
            else if (jj < 0) { jj = -1 - jj; ghost = true; }
            else if (jj >= n) { jj = 2 * n - 1 - jj; ghost = true; }
            const int64_t kk = k + (int64_t)(jj - j) * stride;
            av[s] = a[kk];
            T uu = u[(int64_t)d * r.N + kk];
            if (ghost) uu = -uu;
            wv[s] = vert ? uu - vs : uu;
        }
        int jn = j + 1;
        if (jn >= n) jn -= n;   // periodic neighbour (walls never reach here at the top)
        const T pb = scale * (lam[k + (int64_t)(jn - j) * stride] - lam[k]);
        T fa6[6], fw6[6];
        face_vjp<T>(av, wv, pb, kap, eps, fa6, fw6);
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            fa[base + s * r.N] = fa6[s];
            fw[base + s * r.N] = fw6[s];
        }
    }
}

// ---------------------------------------------------------------------------
// 3. streaming, collision and moments in reverse
// ---------------------------------------------------------------------------
// Reverse of streaming, collision and moments at node k given the node's
// total velocity adjoint ub (transport part included); writes fbar and
// returns the node's contribution to cbar through the force.
template <int Q, typename T, bool SH>
__device__ __forceinline__ T collide_reverse_node(const AdjDev &A, int64_t k, int x, int y, int z,
                                                  const T ubt[3]) {
    using L = Lattice<Q>;
    constexpr int D = L::D;
    const RunDev &r = A.r;
    const T *fbn = (const T *)A.fbar_next;
    T fi[Q], fsb[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // forward streaming sent f*_i(x) to slot i of x + c_i, or to slot
        // opp(i) of x across a wall: pull the adjoint from there
        const int64_t dst = displaced<D>(r, x, y, z, L::cx[i], L::cy[i], L::cz[i]);
        fsb[i] = dst >= 0 ? fbn[(int64_t)i * r.N + dst] : fbn[(int64_t)L::opp[i] * r.N + k];
    }
    T F[3], u[3] = {0, 0, 0}, rho;
    lbm_force<D, T>(r, (const T *)A.c_n, nullptr, k, F);
    if (A.have_rho) {
        // the forward step's own moments (what lbm_rho_u gives from f^n, bit
        // for bit): the populations themselves are not needed
        const T *uu = (const T *)A.u;
#pragma unroll
        for (int d = 0; d < D; ++d) u[d] = uu[(int64_t)d * r.N + k];
        rho = ((const T *)A.rho_n)[k];
    } else {
        const T *f = (const T *)A.f_n;
#pragma unroll
        for (int i = 0; i < Q; ++i) fi[i] = f[(int64_t)i * r.N + k];
        T drho;
        lbm_rho_u<Q, T, SH>(fi, F, rho, drho, u);
    }
    const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T omega = (T)r.omega, guo = (T)r.guo;
    T ub[3] = {ubt[0], ubt[1], ubt[2]}, Fb[3] = {0, 0, 0}, rb = 0;
    T *fb = (T *)A.fbar;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T w = (T)L::w[i];
        const T c[3] = {(T)L::cx[i], (T)L::cy[i], (T)L::cz[i]};
        const T cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        const T cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2];
        const T poly = (T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * usq;
        // f* = f - omega (f - feq(rho, u)) + G(u, F)
        const T eb = omega * fsb[i];      // adjoint of feq_i
        const T gb = fsb[i];              // adjoint of G_i
        rb += eb * w * ((T)1 + poly);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ub[d] += eb * w * rho * ((T)3 * c[d] + (T)9 * cu * c[d] - (T)3 * u[d]) +
                     gb * guo * w * ((T)-3 * F[d] + (T)9 * c[d] * cF);
            Fb[d] += gb * guo * w * ((T)3 * (c[d] - u[d]) + (T)9 * cu * c[d]);
        }
        fi[i] = ((T)1 - omega) * fsb[i];
    }
    // u = (m + F/2) / rho, m = sum f c, rho = sum f (+1 when shifted)
    T mb[3];
    const T irho = rcp<T>(rho);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        mb[d] = ub[d] * irho;
        Fb[d] += (T)0.5 * mb[d];
        rb -= mb[d] * u[d];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        fb[(int64_t)i * r.N + k] = fi[i] + (rb + mb[0] * (T)L::cx[i] + mb[1] * (T)L::cy[i] + mb[2] * (T)L::cz[i]);
    return -(T)r.gp_c * Fb[D - 1];
}

// ---------------------------------------------------------------------------
// gather of the transport transpose (the last reversed stage also reverses
// the collision at the node)
// ---------------------------------------------------------------------------
// Node-wise gather of the face products.  STAGE selects the RK stage being
// reversed (3, 2, 1 in that order) and how the result combines.
// The per-node end of a reversed RK stage, given the node's gathered face
// products (abar, the velocity parts ubs and the settling part vsp): the
// absorbing bottom face, the deposit update, the RK combination and, after the
// last stage, the collision and moments in reverse.
template <int Q, typename T, bool SH, int STAGE>
__device__ __forceinline__ void gather_finish(const AdjDev &A, int64_t k, int x, int y, int z, T abar,
                                              const T ubs[3], double vsp) {
    constexpr int D = Lattice<Q>::D;
    const RunDev &r = A.r;
    T *ub = (T *)A.ubar;
    // bottom wall face: L_0 contains -vs a_0
    const int v = (D == 2) ? y : z;
    const bool bottom = !r.vper && v == 0;
    const T *lam_in;
    T lam_scale;
    const T *a_fwd;
    if constexpr (STAGE == 3) { lam_in = (const T *)A.cbar_next; lam_scale = (T)(2.0 / 3.0); a_fwd = (const T *)A.a2; }
    else if constexpr (STAGE == 2) { lam_in = (const T *)A.abar2; lam_scale = (T)0.25; a_fwd = (const T *)A.a1; }
    else { lam_in = (const T *)A.abar1; lam_scale = (T)1; a_fwd = (const T *)A.c_n; }
    const T lam = lam_scale * lam_in[k];
    if (bottom) {
        abar += -(T)r.vs * lam;
        vsp += -(double)a_fwd[k] * (double)lam;
    }
    const double db = A.dep_bar;
    const T *cbn = (const T *)A.cbar_next;
    T *cb = (T *)A.cbar;
    if constexpr (STAGE == 3) {
        T a2b = (T)(2.0 / 3.0) * cbn[k] + abar;
        T cbv = cbn[k] * (T)(1.0 / 3.0);
        if (bottom) {
            // D+ = D + vs (C/6 + a1/6 + 2 a2/3)
            a2b += (T)(2.0 / 3.0 * r.vs * db);
            cbv += (T)(r.vs / 6.0 * db);
            vsp += db * ((double)((const T *)A.c_n)[k] / 6.0 + (double)((const T *)A.a1)[k] / 6.0 +
                         2.0 / 3.0 * (double)((const T *)A.a2)[k]);
        }
        ((T *)A.abar2)[k] = a2b;
        cb[k] = cbv;
#pragma unroll
        for (int d = 0; d < D; ++d) ub[(int64_t)d * r.N + k] = ubs[d];
        A.vs_part[k] += vsp;      // accumulates across steps until summed
    } else if constexpr (STAGE == 2) {
        const T a2b = ((const T *)A.abar2)[k];
        T a1b = (T)0.25 * a2b + abar;
        if (bottom) a1b += (T)(r.vs / 6.0 * db);
        ((T *)A.abar1)[k] = a1b;
        cb[k] += (T)0.75 * a2b;
#pragma unroll
        for (int d = 0; d < D; ++d) ub[(int64_t)d * r.N + k] += ubs[d];
        A.vs_part[k] += vsp;
    } else {
        T cbv = cb[k] + ((const T *)A.abar1)[k] + abar;
        A.vs_part[k] += vsp;
        if (A.frozen) {
            cb[k] = cbv;
        } else {
            // last stage reversed: the node's velocity adjoint is complete, so
            // the collision and moments are reversed here as well
            T ut[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < D; ++d) ut[d] = ub[(int64_t)d * r.N + k] + ubs[d];
            cb[k] = cbv + collide_reverse_node<Q, T, SH>(A, k, x, y, z, ut);
        }
    }
}

template <int Q, typename T, bool SH, int STAGE>
__global__ void __launch_bounds__(256) k_adj_gather(AdjDev A) {
    constexpr int D = Lattice<Q>::D;
    const RunDev &r = A.r;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= r.N) return;
    int x, y, z;
    xyz<D>(r, k, x, y, z);
    const T *fa = (const T *)A.faceA, *fw = (const T *)A.faceW;
    double vsp = 0.0;
    T abar = 0;
    T ubs[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const bool vert = (d == D - 1);
        const bool walls = vert && !r.vper;
        const int m = d == 0 ? x : (d == 1 ? y : z);
        const int n = d == 0 ? r.nx : (d == 1 ? r.ny : r.nz);
        const int64_t stride = d == 0 ? 1 : (d == 1 ? (int64_t)r.nx : (int64_t)r.nx * r.ny);
        // images of node m as seen by stencils: itself, and beyond each wall
        // (only rows m <= 1 and m >= n - 2 have images that a face reads)
        const int nimg = (walls && (m <= 1 || m >= n - 2)) ? 3 : 1;
        for (int im = 0; im < nimg; ++im) {
            const int p = im == 0 ? m : (im == 1 ? -1 - m : 2 * n - 1 - m);
            const bool ghost = im != 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                int jf = p - s + 2;              // face whose slot s reads position p
                if (walls) {
                    if (jf < 0 || jf > n - 2) continue;
                } else {
                    jf = wrap_near(jf, n);
                }
                const int64_t kf = k + (int64_t)(jf - m) * stride;
                const int64_t idx = ((int64_t)d * 6 + s) * r.N + kf;
                abar += fa[idx];
                const T wb = fw[idx];
                if (vert) {
                    ubs[d] += ghost ? -wb : wb;
                    vsp -= (double)wb;
                } else {
                    ubs[d] += wb;
                }
            }
        }
    }
    gather_finish<Q, T, SH, STAGE>(A, k, x, y, z, abar, ubs, vsp);
}

// ---------------------------------------------------------------------------
// 2D: one reversed RK stage in one kernel.  A block owns a TX x TY tile of
// nodes and keeps everything between the stage's inputs and its per-node
// results in LDS: the stage input a, the transport velocity and the face
// adjoints lam with the halos the tile's face stencils reach (wall images
// already mirrored, with the sign of the vertical velocity flipped); the
// products of every x face the tile's nodes read (five faces beyond the
// tile), gathered per node; then the same for the y faces.  Faces are
// evaluated with the same face_vjp on the same values as the two-kernel form
// and gathered in the same order, so the results are identical bit for bit;
// the workspace round trip of the face products disappears, at the price of
// recomputing the five faces per row and column that neighbouring tiles also
// need.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_any(int j, int n) {
    j %= n;
    return j < 0 ? j + n : j;
}

template <typename T, bool SH, int STAGE, int TX, int TY>
__global__ void __launch_bounds__(256) k_adj_stage2d(AdjDev A, const T *__restrict__ a,
                                                     const T *__restrict__ lam, T scale) {
    constexpr int NT = 256, PER = TX * TY / NT;
    static_assert(TX * TY % NT == 0, "tile must be a multiple of the block");
    constexpr int HX = TX + 10, LX = TX + 6, NFX = TX + 5;   // x: a/w row, lam row, faces per row
    constexpr int HY = TY + 10, LY = TY + 6, NFY = TY + 5;   // y: the same per column
    constexpr int NP = (NFX * TY > NFY * TX) ? NFX * TY : NFY * TX;
    __shared__ T sAx[TY * HX], sWx[TY * HX], sLx[TY * LX];
    __shared__ T sAy[HY * TX], sWy[HY * TX], sLy[LY * TX];
    __shared__ T sPA[6 * NP], sPW[6 * NP];

    const RunDev &r = A.r;
    const int nx = r.nx, ny = r.ny;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tid = threadIdx.x;
    const bool walls = !r.vper;
    const T *u = (const T *)(A.frozen ? r.u : A.u);
    const T *ux = u, *uy = u + r.N;
    const T vs = (T)r.vs, kap = (T)r.kappa_c, eps = (T)r.eps;
    // vertical position p of a stencil or lam row -> stored row (mirrored
    // beyond walls; rows no face of the tile reads are clamped into range)
    auto vrow = [&](int p, bool &ghost) {
        ghost = false;
        if (!walls) return wrap_any(p, ny);
        if (p < 0) { p = -1 - p; ghost = true; }
        else if (p >= ny) { p = 2 * ny - 1 - p; ghost = true; }
        return p < 0 ? 0 : (p >= ny ? ny - 1 : p);
    };

    // stage the inputs.  Every slot is loaded into registers first,
    // unconditionally (a spare slot repeats the last entry of its array), so
    // all of the tile's loads are in flight together; a loop that stored
    // each load to LDS before issuing the next waited for every load in turn
    constexpr int N1 = TY * HX, N2 = TY * LX, N3 = HY * TX, N4 = LY * TX;
    constexpr int S1 = (N1 + NT - 1) / NT, S2 = (N2 + NT - 1) / NT, S3 = (N3 + NT - 1) / NT,
                  S4 = (N4 + NT - 1) / NT;
    T pA1[S1], pW1[S1], pL2[S2], pA3[S3], pW3[S3], pL4[S4];
    bool g3[S3];
#pragma unroll
    for (int q = 0; q < S1; ++q) {
        const int i = min(tid + q * NT, N1 - 1);
        const int ly = i / HX, c = i % HX;
        const int gy = min(y0 + ly, ny - 1);
        const int64_t k = (int64_t)wrap_any(x0 - 5 + c, nx) + (int64_t)nx * gy;
        pA1[q] = a[k];
        pW1[q] = ux[k];
    }
#pragma unroll
    for (int q = 0; q < S2; ++q) {
        const int i = min(tid + q * NT, N2 - 1);
        const int ly = i / LX, c = i % LX;
        const int gy = min(y0 + ly, ny - 1);
        pL2[q] = lam[(int64_t)wrap_any(x0 - 3 + c, nx) + (int64_t)nx * gy];
    }
#pragma unroll
    for (int q = 0; q < S3; ++q) {
        const int i = min(tid + q * NT, N3 - 1);
        const int ry = i / TX, lx = i % TX;
        const int gy = vrow(y0 - 5 + ry, g3[q]);
        const int64_t k = (int64_t)wrap_any(x0 + lx, nx) + (int64_t)nx * gy;
        pA3[q] = a[k];
        pW3[q] = uy[k];
    }
#pragma unroll
    for (int q = 0; q < S4; ++q) {
        const int i = min(tid + q * NT, N4 - 1);
        const int ry = i / TX, lx = i % TX;
        bool ghost;
        const int gy = vrow(y0 - 3 + ry, ghost);
        pL4[q] = lam[(int64_t)wrap_any(x0 + lx, nx) + (int64_t)nx * gy];
    }
#pragma unroll
    for (int q = 0; q < S1; ++q) {
        const int i = tid + q * NT;
        if (i < N1) { sAx[i] = pA1[q]; sWx[i] = pW1[q]; }
    }
#pragma unroll
    for (int q = 0; q < S2; ++q) {
        const int i = tid + q * NT;
        if (i < N2) sLx[i] = pL2[q];
    }
#pragma unroll
    for (int q = 0; q < S3; ++q) {
        const int i = tid + q * NT;
        if (i < N3) { sAy[i] = pA3[q]; sWy[i] = (g3[q] ? -pW3[q] : pW3[q]) - vs; }
    }
#pragma unroll
    for (int q = 0; q < S4; ++q) {
        const int i = tid + q * NT;
        if (i < N4) sLy[i] = pL4[q];
    }
    __syncthreads();

    // x faces j = x0 - 3 + i of every tile row (the x axis is periodic)
    for (int f = tid; f < NFX * TY; f += NT) {
        const int ly = f / NFX, i = f % NFX;
        T av[6], wv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            av[q] = sAx[ly * HX + i + q];
            wv[q] = sWx[ly * HX + i + q];
        }
        const T pb = scale * (sLx[ly * LX + i + 1] - sLx[ly * LX + i]);
        T fa6[6], fw6[6];
        face_vjp<T>(av, wv, pb, kap, eps, fa6, fw6);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            sPA[q * NP + f] = fa6[q];
            sPW[q * NP + f] = fw6[q];
        }
    }
    __syncthreads();
    T abar[PER], ubx[PER], uby[PER];
    double vsp[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int node = tid + e * NT, lx = node % TX, ly = node / TX;
        abar[e] = 0;
        ubx[e] = 0;
        uby[e] = 0;
        vsp[e] = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {            // face x - q + 2 reads this node at slot q
            const int f = ly * NFX + lx + 5 - q;
            abar[e] += sPA[q * NP + f];
            ubx[e] += sPW[q * NP + f];
        }
    }
    __syncthreads();

    // y faces j = y0 - 3 + i of every tile column (faces exist for
    // 0 <= j <= ny - 2 with walls; periodic positions wrap)
    for (int f = tid; f < NFY * TX; f += NT) {
        const int iy = f / TX, lx = f % TX;
        const int j = y0 - 3 + iy;
        if (walls && (j < 0 || j > ny - 2)) continue;   // never gathered
        T av[6], wv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            av[q] = sAy[(iy + q) * TX + lx];
            wv[q] = sWy[(iy + q) * TX + lx];
        }
        const T pb = scale * (sLy[(iy + 1) * TX + lx] - sLy[iy * TX + lx]);
        T fa6[6], fw6[6];
        face_vjp<T>(av, wv, pb, kap, eps, fa6, fw6);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            sPA[q * NP + f] = fa6[q];
            sPW[q * NP + f] = fw6[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int node = tid + e * NT, lx = node % TX, ly = node / TX;
        const int m = y0 + ly;
        // only nodes of the grid gather: for a row beyond the top of a ragged
        // tile the image above the wall could name a face outside the tile's
        // range.  For a grid node every face it reads lies in [y0 - 3, y0 + TY + 1]:
        // its own faces m - 3 .. m + 2, the bottom images (faces 0, 1, read only
        // when m <= 1, so y0 = 0) and the top images (faces >= ny - 3 >= m - 2,
        // read only when m >= ny - 3).
        if (x0 + lx >= nx || m >= ny) continue;
        // wall images reach only rows m <= 1 (the image -1 - m feeds faces 0
        // and 1) and m >= ny - 2 (the image 2 ny - 1 - m feeds faces ny - 3
        // and ny - 2); tiles clear of both take the node itself only (the
        // same sum: the skipped images add nothing)
        const int nimg = (walls && (y0 < 2 || y0 + TY > ny - 2)) ? 3 : 1;
        for (int im = 0; im < nimg; ++im) {
            const int p = im == 0 ? m : (im == 1 ? -1 - m : 2 * ny - 1 - m);
            const bool ghost = im != 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int jf = p - q + 2;        // face whose slot q reads position p
                if (walls && (jf < 0 || jf > ny - 2)) continue;
                const int f = (jf - (y0 - 3)) * TX + lx;
                abar[e] += sPA[q * NP + f];
                const T wb = sPW[q * NP + f];
                uby[e] += ghost ? -wb : wb;
                vsp[e] -= (double)wb;
            }
        }
        const int64_t k = (int64_t)(x0 + lx) + (int64_t)nx * m;
        const T ubs[3] = {ubx[e], uby[e], (T)0};
        gather_finish<9, T, SH, STAGE>(A, k, x0 + lx, m, 0, abar[e], ubs, vsp[e]);
    }
}

// ---------------------------------------------------------------------------
// dJ/dVs: fixed-order FP64 sum of the per-node parts, added to *vs_bar
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_adj(double acc) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double waves[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) waves[wid] = acc;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); ++i) t += waves[i];
    return t;
}

__global__ void __launch_bounds__(256) k_adj_vs_partial(double *__restrict__ part, int64_t n,
                                                        double *__restrict__ out) {
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        acc += part[k];
        part[k] = 0.0;            // the accumulator starts over
    }
    const double t = block_sum_adj(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_adj_vs_final(const double *__restrict__ part, int n,
                                                      double *__restrict__ vs_bar) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    const double t = block_sum_adj(acc);
    if (threadIdx.x == 0) *vs_bar += t;
}

template <int Q, typename T, bool SH>
hipError_t adjoint_t(const AdjDev &A, const lbw_launch &l, hipStream_t st) {
    constexpr int D = Lattice<Q>::D;
    const int block = 256;
    const dim3 grid((unsigned)((A.r.N + block - 1) / block));
    if (!A.frozen && !A.have_u) k_adj_moments<Q, T, SH><<<grid, block, 0, st>>>(A);
    hipError_t e = hipSuccess;
    if (!A.have_stages) {
        // forward stages 1 and 2 from the saved C^n and u^n, with the same
        // tiled kernels as the forward step (a1, a2 are its own values)
        RunDev fr = A.r;
        fr.c = const_cast<void *>(A.c_n);
        fr.c1 = A.a1;
        fr.c2 = A.a2;
        fr.u = A.frozen ? A.r.u : A.u;
        const int prec = sizeof(T) == 4 ? LBW_FP32_SHIFTED : LBW_FP64;
        lbw_launch lt = l;
        lt.variant = 0;
        // one block per tile and chunk, fewer than 2^32 work-items a launch
        const TileShape sh = resolve_tile_shape(D, lt);
        if (transport_tiles(D, fr, lt) * sh.tx * sh.ty >= ((int64_t)1 << 32)) return hipErrorInvalidConfiguration;
        e = launch_one_stage(D, prec, fr, lt, 1, st);
        if (e == hipSuccess) e = launch_one_stage(D, prec, fr, lt, 2, st);
        if (e != hipSuccess) return e;
    }
    // the fused 2D form launches one block row per TY grid rows; a launch
    // takes at most 65535 block rows, so taller runs take the two-kernel form
    // (the same sums in the same order: the same bits)
    constexpr int TX = sizeof(T) == 4 ? 32 : 16, TY = sizeof(T) == 4 ? 8 : 16;
    const int64_t block_rows = ((int64_t)A.r.ny + TY - 1) / TY;
    if (D == 2 && l.variant != 1 && block_rows <= 65535) {
        // one kernel per reversed stage, face products kept in LDS
        const dim3 tg((unsigned)((A.r.nx + TX - 1) / TX), (unsigned)block_rows);
        k_adj_stage2d<T, SH, 3, TX, TY><<<tg, 256, 0, st>>>(A, (const T *)A.a2, (const T *)A.cbar_next, (T)(2.0 / 3.0));
        k_adj_stage2d<T, SH, 2, TX, TY><<<tg, 256, 0, st>>>(A, (const T *)A.a1, (const T *)A.abar2, (T)0.25);
        k_adj_stage2d<T, SH, 1, TX, TY><<<tg, 256, 0, st>>>(A, (const T *)A.c_n, (const T *)A.abar1, (T)1);
    } else {
        k_adj_face<T, D><<<grid, block, 0, st>>>(A, (const T *)A.a2, (const T *)A.cbar_next, (T)(2.0 / 3.0));
        k_adj_gather<Q, T, SH, 3><<<grid, block, 0, st>>>(A);
        k_adj_face<T, D><<<grid, block, 0, st>>>(A, (const T *)A.a1, (const T *)A.abar2, (T)0.25);
        k_adj_gather<Q, T, SH, 2><<<grid, block, 0, st>>>(A);
        k_adj_face<T, D><<<grid, block, 0, st>>>(A, (const T *)A.c_n, (const T *)A.abar1, (T)1);
        k_adj_gather<Q, T, SH, 1><<<grid, block, 0, st>>>(A);
    }
    if (A.vs_bar) {
        k_adj_vs_partial<<<kReduceBlocks, 256, 0, st>>>(A.vs_part, A.r.N, A.partials);
        k_adj_vs_final<<<1, 256, 0, st>>>(A.partials, kReduceBlocks, A.vs_bar);
    }
    return hipGetLastError();
}

}  // namespace

size_t adjoint_work_bytes(int dim, int precision, int64_t N) {
    const size_t es = precision == LBW_FP32_SHIFTED ? 4 : 8;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t b = 0;
    b += al(es * dim * N);          // u
    b += 4 * al(es * N);            // a1, a2, abar1, abar2
    b += al(es * dim * N);          // ubar
    b += 2 * al(es * 6 * dim * N);  // face products
    b += al(sizeof(double) * N);    // vs parts
    b += al(sizeof(double) * kReduceBlocks);
    return b;
}

hipError_t launch_adjoint(int q, int precision, const RunDev &r, bool frozen, const void *f_n,
                          const void *c_n, const void *u_n, const void *rho_n, const void *a1_n,
                          const void *a2_n,
                          const void *fbar_next, const void *cbar_next,
                          double dep_bar, void *fbar, void *cbar, double *vs_bar, void *work,
                          const lbw_launch &l, hipStream_t st) {
    const int dim = q == 9 ? 2 : 3;
    const size_t es = precision == LBW_FP32_SHIFTED ? 4 : 8;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char *w = (char *)work;
    AdjDev A;
    A.r = r;
    A.f_n = f_n;
    A.c_n = c_n;
    A.rho_n = rho_n;
    A.fbar_next = fbar_next;
    A.cbar_next = cbar_next;
    A.fbar = fbar;
    A.cbar = cbar;
    A.u = w; w += al(es * dim * r.N);
    A.a1 = w; w += al(es * r.N);
    A.a2 = w; w += al(es * r.N);
    A.abar1 = w; w += al(es * r.N);
    A.abar2 = w; w += al(es * r.N);
    A.ubar = w; w += al(es * dim * r.N);
    A.faceA = w; w += al(es * 6 * dim * r.N);
    A.faceW = w; w += al(es * 6 * dim * r.N);
    A.vs_part = (double *)w; w += al(sizeof(double) * r.N);
    A.partials = (double *)w;
    A.vs_bar = vs_bar;
    A.dep_bar = dep_bar;
    A.frozen = frozen ? 1 : 0;
    A.have_u = (u_n != nullptr && !frozen) ? 1 : 0;
    A.have_rho = (A.have_u && rho_n != nullptr) ? 1 : 0;
    A.have_stages = (a1_n != nullptr && a2_n != nullptr) ? 1 : 0;
    if (A.have_u) A.u = const_cast<void *>(u_n);
    if (A.have_stages) {
        A.a1 = const_cast<void *>(a1_n);
        A.a2 = const_cast<void *>(a2_n);
    }
    switch (precision) {
        case LBW_FP64: return q == 9 ? adjoint_t<9, double, false>(A, l, st) : adjoint_t<19, double, false>(A, l, st);
        case LBW_FP64_SHIFTED: return q == 9 ? adjoint_t<9, double, true>(A, l, st) : adjoint_t<19, double, true>(A, l, st);
        case LBW_FP32_SHIFTED: return q == 9 ? adjoint_t<9, float, true>(A, l, st) : adjoint_t<19, float, true>(A, l, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbw
