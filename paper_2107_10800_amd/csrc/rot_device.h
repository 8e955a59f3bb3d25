// Generalised RPY tensor of single-blob bodies (Sec. 2.4), device helpers shared
// by the dense product (rot_pair.hip) and the fast product (fmm.hip).  With
// r = x_i - x_j, in units of 1/(8 pi eta):
//     u_i += c1 f_j + c2 (r . f_j) r + c_r tau_j x r
//     w_i += c_r f_j x r + d1 tau_j + d2 (r . tau_j) r
// (coefficients and their overlap branch: see rot_pair.hip).
#pragma once
#include "rpy_device.h"

namespace arb {

template <class T>
struct RotCoef {
    T k1, k2, n1, n2, n3, four_a2, e1, e2, g0, g1, g3, h1, h3;
};

inline RotCoef<double> rot_coef(double a) {
    RotCoef<double> c;
    const double a2 = a * a, a3 = a2 * a, a4 = a2 * a2, a6 = a3 * a3;
    c.k1 = 2.0 * a2 / 3.0;
    c.k2 = 2.0 * a2;
    c.n1 = 4.0 / (3.0 * a);
    c.n2 = 3.0 / (8.0 * a2);
    c.n3 = 1.0 / (8.0 * a2);
    c.four_a2 = 4.0 * a2;
    c.e1 = 1.0 / (2.0 * a3);
    c.e2 = 3.0 / (16.0 * a4);
    c.g0 = 1.0 / a3;
    c.g1 = 27.0 / (32.0 * a4);
    c.g3 = 5.0 / (64.0 * a6);
    c.h1 = 9.0 / (32.0 * a4);
    c.h3 = 3.0 / (64.0 * a6);
    return c;
}

// a = 1 (the FP32 kernels)
constexpr RotCoef<float> kUnitRotCoef{2.f / 3.f,  2.f,        4.f / 3.f,  3.f / 8.f,   1.f / 8.f,
                                      4.f,        0.5f,       3.f / 16.f, 1.f,         27.f / 32.f,
                                      5.f / 64.f, 9.f / 32.f, 3.f / 64.f};

template <class T>
struct RotTerms {
    T c1, c2, cr, d1, d2;
};

// rinv = 1/sqrt(r2), not finite at r = 0 (that case takes the overlap branch)
template <class T>
__device__ __forceinline__ RotTerms<T> rot_terms(T r2, T rinv, const RotCoef<T> &c) {
    RotTerms<T> k;
    const T rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
    k.c1 = fma(c.k1, rinv3, rinv);
    k.c2 = fma(-c.k2, rinv3 * rinv2, rinv3);
    k.cr = rinv3;
    k.d1 = T(-0.5) * rinv3;
    k.d2 = T(1.5) * rinv3 * rinv2;
    ARB_IF_ANY_OVERLAP(r2 <= c.four_a2)
    if (r2 <= c.four_a2) {
        const T rv = r2 > T(0) ? rinv : T(0);
        const T r = r2 * rv;
        k.c1 = fma(-c.n2, r, c.n1);
        k.c2 = rv * c.n3;
        k.cr = fma(-c.e2, r, c.e1);
        k.d1 = fma(r, fma(c.g3, r * r, -c.g1), c.g0);
        k.d2 = fma(c.h1, rv, -c.h3 * r);
    }
    ARB_END_IF_ANY
    return k;
}

// a += N_ij (f, t) for r = (dx, dy, dz); c_r applied to r once for both cross
// products
template <class T>
__device__ __forceinline__ void rot_one_way(const RotTerms<T> &k, T dx, T dy, T dz, T fx, T fy,
                                            T fz, T tx, T ty, T tz, T *a) {
    const T tf = k.c2 * fma(dx, fx, fma(dy, fy, dz * fz));
    const T tt = k.d2 * fma(dx, tx, fma(dy, ty, dz * tz));
    const T ex = k.cr * dx, ey = k.cr * dy, ez = k.cr * dz;
    a[0] = fma(k.c1, fx, fma(tf, dx, fma(ty, ez, fma(-tz, ey, a[0]))));
    a[1] = fma(k.c1, fy, fma(tf, dy, fma(tz, ex, fma(-tx, ez, a[1]))));
    a[2] = fma(k.c1, fz, fma(tf, dz, fma(tx, ey, fma(-ty, ex, a[2]))));
    a[3] = fma(k.d1, tx, fma(tt, dx, fma(fy, ez, fma(-fz, ey, a[3]))));
    a[4] = fma(k.d1, ty, fma(tt, dy, fma(fz, ex, fma(-fx, ez, a[4]))));
    a[5] = fma(k.d1, tz, fma(tt, dz, fma(fx, ey, fma(-fy, ex, a[5]))));
}

}  // namespace arb
