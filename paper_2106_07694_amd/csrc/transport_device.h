// transport_device.h -- face fluxes of the scalar transport (supplement
// section 1): WENO reconstruction of the advective flux h = w a from the
// upwind side of each face, central diffusion, and the wall rules.
#pragma once

#include "lbw_internal.h"

namespace lbw {

// WENO5-JS (Jiang & Shu 1996, the fifth-order member of the family the
// supplement's S8-S16 introduce): value at the downwind face of the centre of
// five nodes ordered upwind -> downwind.  Candidates use the node fluxes h,
// smoothness indicators the transported values a.
template <typename T>
__device__ __forceinline__ T weno5_face(T h0, T h1, T h2, T h3, T h4, T a0, T a1, T a2, T a3,
                                        T a4, T eps) {
    const T q0 = ((T)2 * h0 - (T)7 * h1 + (T)11 * h2) * (T)(1.0 / 6.0);
    const T q1 = (-h1 + (T)5 * h2 + (T)2 * h3) * (T)(1.0 / 6.0);
    const T q2 = ((T)2 * h2 + (T)5 * h3 - h4) * (T)(1.0 / 6.0);
    T t = a0 - (T)2 * a1 + a2, s = a0 - (T)4 * a1 + (T)3 * a2;
    const T b0 = (T)(13.0 / 12.0) * t * t + (T)0.25 * s * s;
    t = a1 - (T)2 * a2 + a3;
    s = a1 - a3;
    const T b1 = (T)(13.0 / 12.0) * t * t + (T)0.25 * s * s;
    t = a2 - (T)2 * a3 + a4;
    s = (T)3 * a2 - (T)4 * a3 + a4;
    const T b2 = (T)(13.0 / 12.0) * t * t + (T)0.25 * s * s;
    const T e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
    const T al0 = (T)0.1 / (e0 * e0);
    const T al1 = (T)0.6 / (e1 * e1);
    const T al2 = (T)0.3 / (e2 * e2);
    return (al0 * q0 + al1 * q1 + al2 * q2) / (al0 + al1 + al2);
}

// WENO3 (S10-S16): upwind two-node candidate (S11) weighted 1/3, central
// candidate (S10) weighted 2/3; nodes ordered upwind -> downwind.
template <typename T>
__device__ __forceinline__ T weno3_face(T h0, T h1, T h2, T a0, T a1, T a2, T eps) {
    const T qu = (T)0.5 * ((T)3 * h1 - h0);
    const T qc = (T)0.5 * (h1 + h2);
    const T eu = eps + (a1 - a0) * (a1 - a0);
    const T ec = eps + (a2 - a1) * (a2 - a1);
    const T au = (T)(1.0 / 3.0) / (eu * eu);
    const T ac = (T)(2.0 / 3.0) / (ec * ec);
    return (au * qu + ac * qc) / (au + ac);
}

// Total flux through the face j+1/2 from the six nodes j-2 .. j+3 (values a,
// transport velocities w): reconstructed advective flux from the side the
// face velocity (w_j + w_{j+1})/2 comes from (ties count as positive), minus
// kappa times the central difference.
template <typename T, int SCHEME>
__device__ __forceinline__ T face_flux(const T *a, const T *w, T kappa, T eps) {
    const T wf = (T)0.5 * (w[2] + w[3]);
    T hh;
    if constexpr (SCHEME == LBW_WENO5) {
        if (wf >= (T)0)
            hh = weno5_face<T>(w[0] * a[0], w[1] * a[1], w[2] * a[2], w[3] * a[3], w[4] * a[4],
                               a[0], a[1], a[2], a[3], a[4], eps);
        else
            hh = weno5_face<T>(w[5] * a[5], w[4] * a[4], w[3] * a[3], w[2] * a[2], w[1] * a[1],
                               a[5], a[4], a[3], a[2], a[1], eps);
    } else if constexpr (SCHEME == LBW_WENO3) {
        if (wf >= (T)0)
            hh = weno3_face<T>(w[1] * a[1], w[2] * a[2], w[3] * a[3], a[1], a[2], a[3], eps);
        else
            hh = weno3_face<T>(w[4] * a[4], w[3] * a[3], w[2] * a[2], a[4], a[3], a[2], eps);
    } else {
        hh = (wf >= (T)0) ? w[2] * a[2] : w[3] * a[3];
    }
    return hh - kappa * (a[3] - a[2]);
}

// Combinations of the second and third RK3 stages (S22, S23), given the
// base value c, the stage input a and its right-hand side L:
//   3/4 c + 1/4 a + 1/4 L  and  1/3 c + 2/3 a + 2/3 L,
// written as c plus a small increment.  The stage input differs from c by
// O(L), so a - c is exact when the two are within a factor of two, and the
// stored value takes one rounding, at the final add; summing the weighted
// terms directly rounds each product of an O(1) value and each partial sum,
// which in single precision is the leading error of the transported field.
template <typename T>
__device__ __forceinline__ T rk3_stage2(T c, T a, T L) {
    return c + (T)0.25 * ((a - c) + L);
}
template <typename T>
__device__ __forceinline__ T rk3_stage3(T c, T a, T L) {
    return c + (T)(2.0 / 3.0) * ((a - c) + L);
}

}  // namespace lbw
