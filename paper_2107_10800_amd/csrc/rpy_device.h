// RPY pair tensor device code shared by the mat-vec and the preconditioner
// assembly (Sec. 2.3, Eq. RPY); see pair.hip for the formulas.
#pragma once
#include "common.h"

namespace arb {

struct CoefF {
    float k1, k2, n1, n2, n3, a2, four_a2, a4;
};
struct CoefD {
    double k1, k2, n1, n2, n3, a2, four_a2, a4;
};

template <class C, class T>
__host__ __device__ inline C make_coef(T a) {
    C c;
    c.k1 = T(2) * a * a / T(3);
    c.k2 = T(2) * a * a;
    c.n1 = T(4) / (T(3) * a);
    c.n2 = T(3) / (T(8) * a * a);
    c.n3 = T(1) / (T(8) * a * a);
    c.a2 = a * a;
    c.four_a2 = T(4) * a * a;
    c.a4 = a * a * a * a;
    return c;
}

// Coefficients for a = 1.  The FP32 kernels work in units of the blob radius
// (positions divided by a on upload, M(a) = M_{a=1}(r / a) / a): every
// coefficient is then a compile-time literal rather than a kernel argument.
constexpr CoefF kUnitCoefF{2.f / 3.f, 2.f, 4.f / 3.f, 3.f / 8.f, 1.f / 8.f, 1.f, 4.f, 1.f};

__device__ __forceinline__ float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }

// Overlapping pairs (r <= 2a) are rare away from a body's own blobs, so the
// overlap coefficients are computed only when some lane of the wavefront has
// one: a wave vote and a real branch.  The empty volatile asm keeps the branch
// (speculated, the overlap path would be paid by every pair as selects).
#define ARB_IF_ANY_OVERLAP(cond) \
    if (__any(cond)) {           \
        asm volatile("" ::: "memory");
#define ARB_END_IF_ANY }

// accumulate M_free(r) lambda (units 1/(8 pi eta)); rinv = 1/sqrt(r2), infinite at r = 0
template <class T, class C>
__device__ __forceinline__ void rpy_free(T dx, T dy, T dz, T r2, T rinv, T lx, T ly, T lz,
                                         const C &c, T &ax, T &ay, T &az) {
    const T rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
    T c1 = fma(c.k1, rinv3, rinv);            // (1 + k1/r^2)/r
    T c2 = fma(-c.k2, rinv3 * rinv2, rinv3);  // (1 - k2/r^2)/r^3
    ARB_IF_ANY_OVERLAP(r2 <= c.four_a2)
    if (r2 <= c.four_a2) {
        const T rv = r2 > T(0) ? rinv : T(0);  // rinv = 1/sqrt(0) = inf for coincident blobs
        c1 = fma(-c.n2, r2 * rv, c.n1);
        c2 = rv * c.n3;
    }
    ARB_END_IF_ANY
    T rl = fma(dx, lx, fma(dy, ly, dz * lz));
    T t = c2 * rl;
    ax = fma(c1, lx, fma(t, dx, ax));
    ay = fma(c1, ly, fma(t, dy, ay));
    az = fma(c1, lz, fma(t, dz, az));
}

// Free-space tensor plus wall image of one pair, written for reuse in both
// directions.  With d = x_i - x_j, R = (dx, dy, z_i + z_j), h = z_j, Ri = 1/|R|,
// e = R Ri, p = a^2 Ri^2 and the image I = Ri [A^ delta + B^ e e^T + C^ e z^T +
// D^ z e^T + E^ z z^T] (units 1/(8 pi eta)), every coefficient is a polynomial in
// s = Ri^2, t = (e.z)^2 and q = z_i z_j: for instance h/|R| (h/|R| - e.z) = -s q.
// (t is formed as 1 - (dx^2 + dy^2) s, q through pre-scaled target heights.)
// Absorbing the powers of Ri gives
//   M_ij l = (c1 + a) l + (c2 (d.l)) d + (b (R.l) + c l_z) R + (d' (R.l) + e l_z) z
// with a = Ri A^, b = Ri^3 B^, c = Ri^2 C^, d' = Ri^2 D^, e = Ri E^ and the free
// part c1 delta + c2 d d^T; M_ji = M_ij^T uses the same numbers with c and d'
// swapped.  The free part and the image then share the in-plane dot product
// and the l term.
template <class T>
struct PairCoef {
    T cA, cAe, c2, b, c, d, e, h2;  // cAe = cA + e (the z row)
};

// Target-side heights scaled once per target: zs = (-2 zi, 6 zi, -12 zi), so that the
// q = zi zj terms of the image coefficients are single FMAs with zj.
template <class T>
struct TargetZ {
    T a, b, c;
};
template <class T>
__device__ __forceinline__ TargetZ<T> target_z(T zi) {
    return TargetZ<T>{T(-2) * zi, T(6) * zi, T(-12) * zi};
}

// rinv = 1/sqrt(r2) (infinite for coincident blobs), dxy2 = dx^2 + dy^2,
// zs = target_z(zi), h2 = 2 zj, mh22 = -h2^2, Rz = zi + zj, Ri = 1/|R|
// NEAR = false: the caller guarantees r > 2a for every lane (well-separated tiles),
// so the overlap branch and its wave vote are left out
template <class T, class C, bool NEAR = true>
__device__ __forceinline__ PairCoef<T> wall_pair_coef(T r2, T rinv, T dxy2, const TargetZ<T> &zs,
                                                      T zj, T h2, T mh22, T Rz, T Ri,
                                                      const C &k) {
    PairCoef<T> w;
    const T rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
    T c1 = fma(k.k1, rinv3, rinv);
    T c2 = fma(-k.k2, rinv3 * rinv2, rinv3);
    if (NEAR) {
        ARB_IF_ANY_OVERLAP(r2 <= k.four_a2)
        if (r2 <= k.four_a2) {
            const T rv = r2 > T(0) ? rinv : T(0);
            c1 = fma(-k.n2, r2 * rv, k.n1);
            c2 = rv * k.n3;
        }
        ARB_END_IF_ANY
    }
    const T s = Ri * Ri;
    const T Ri3 = Ri * s;
    const T Ri5 = Ri3 * s;
    const T t = fma(-dxy2, s, T(1));  // (e.z)^2 = Rz^2 / R^2 = 1 - dxy2 / R^2
    const T a4s = k.a4 * s;
    const T RzRi5 = Rz * Ri5;
    const T h2Ri3 = h2 * Ri3;
    const T a2 = k.a2;
    const T iA = fma(a4s, fma(T(-10.0 / 3.0), t, T(2.0 / 3.0)),
                     fma(T(2) * a2, t, fma(zs.a, zj, T(-2.0 / 3.0) * a2)));
    const T iB = fma(a4s, fma(T(70.0 / 3.0), t, T(-10.0 / 3.0)),
                     fma(T(-10) * a2, t, fma(zs.b, zj, T(2) * a2)));
    const T iC = fma(a4s, fma(T(-140.0 / 3.0), t, T(40.0 / 3.0)),
                     fma(T(20) * a2, t, fma(zs.c, zj, T(-4) * a2)));
    const T iE = fma(a4s, fma(T(20), t, T(-8.0 / 3.0)), fma(T(-4) * a2, t, mh22));
    w.cA = c1 + fma(Ri3, iA, -Ri);
    w.c2 = c2;
    w.b = fma(Ri5, iB, -Ri3);
    w.c = fma(RzRi5, iC, h2Ri3);
    w.d = fma(T(-20.0 / 3.0) * k.a4, RzRi5 * s, h2Ri3);
    w.e = Ri3 * iE;
    w.cAe = w.cA + w.e;
    w.h2 = h2;
    return w;
}

// f += M l for the pair coefficients w; pass (w.c, w.d) for M_ij and (w.d, w.c)
// for M_ij^T.  The z row uses R_z = d_z + 2 h.
template <class T>
__device__ __forceinline__ void wall_pair_apply(const PairCoef<T> &w, T cc, T dd, T dx, T dy,
                                                T dz, T Rz, T lx, T ly, T lz, T &fx, T &fy,
                                                T &fz) {
    const T dxy = fma(dx, lx, dy * ly);
    const T Sd = fma(dz, lz, dxy);
    const T SR = fma(Rz, lz, dxy);
    const T g = fma(w.b, SR, cc * lz);
    const T tg = fma(w.c2, Sd, g);
    fx = fma(w.cA, lx, fma(tg, dx, fx));
    fy = fma(w.cA, ly, fma(tg, dy, fy));
    fz = fma(w.cAe, lz, fma(tg, dz, fma(g, w.h2, fma(dd, SR, fz))));
}

__device__ __forceinline__ double rsq_f64(double x) {
    // hardware estimate refined by two Newton-Raphson steps for 1/sqrt(x):
    // y <- y + y/2 (1 - x y^2), each step doubling the correct bits
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
}


// 3x3 block M(x, y) / (1/(8 pi eta)) in double, row-major, by contracting with e_x, e_y, e_z
__device__ inline void rpy_block_f64(double dx, double dy, double dz, double zt, double zs,
                                     bool wall, const CoefD &c, double *B) {
    const double dxy2 = fma(dx, dx, dy * dy);
    const double r2 = fma(dz, dz, dxy2);
    const double rinv = rsq_f64(r2);
    const double Rz = zt + zs;
    PairCoef<double> w{};
    if (wall)
        w = wall_pair_coef<double>(r2, rinv, dxy2, target_z(zt), zs, zs + zs, -4.0 * zs * zs, Rz,
                                   rsq_f64(fma(Rz, Rz, dxy2)), c);
    for (int col = 0; col < 3; ++col) {
        const double lx = col == 0, ly = col == 1, lz = col == 2;
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (wall)
            wall_pair_apply<double>(w, w.c, w.d, dx, dy, dz, Rz, lx, ly, lz, ax, ay, az);
        else
            rpy_free<double>(dx, dy, dz, r2, rinv, lx, ly, lz, c, ax, ay, az);
        B[col] = ax;
        B[3 + col] = ay;
        B[6 + col] = az;
    }
}

}  // namespace arb
