// RPY pair tensor device code shared by the mat-vec and the preconditioner
// assembly (Sec. 2.3, Eq. RPY); see pair.hip for the formulas.
#pragma once
#include "common.h"

namespace arb {

struct CoefF {
    float k1, k2, n1, n2, n3, a2, four_a2;
};
struct CoefD {
    double k1, k2, n1, n2, n3, a2, four_a2;
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
    return c;
}

__device__ __forceinline__ float rsq_f32(float x) { return __builtin_amdgcn_rsqf(x); }

// accumulate M_free(r) lambda (units 1/(8 pi eta))
template <class T, class C>
__device__ __forceinline__ void rpy_free(T dx, T dy, T dz, T r2, T rinv, T lx, T ly, T lz,
                                         const C &c, T &ax, T &ay, T &az) {
    T rinv2 = rinv * rinv;
    T c1 = rinv * fma(c.k1, rinv2, T(1));
    T c2 = rinv * rinv2 * fma(-c.k2, rinv2, T(1));
    if (r2 <= c.four_a2) {
        T r = r2 * rinv;
        c1 = fma(-c.n2, r, c.n1);
        c2 = rinv * c.n3;
    }
    T rl = fma(dx, lx, fma(dy, ly, dz * lz));
    T t = c2 * rl;
    ax = fma(c1, lx, fma(t, dx, ax));
    ay = fma(c1, ly, fma(t, dy, ay));
    az = fma(c1, lz, fma(t, dz, az));
}

// accumulate the wall image I(x, y) lambda; dx, dy in-plane target-source,
// Rz = target height + source height, h = source height, Ri = 1/|R|
template <class T, class C>
__device__ __forceinline__ void rpy_image(T dx, T dy, T Rz, T h, T Ri, T lx, T ly, T lz,
                                          const C &c, T &ax, T &ay, T &az) {
    const T e3 = Rz * Ri;
    const T hh = h * Ri;
    const T Ri2 = Ri * Ri;
    const T p = c.a2 * Ri2;
    const T p2 = p * p;
    const T e32 = e3 * e3;
    const T hh2 = hh * hh;
    const T eh = e3 * hh;
    T Ah = fma(T(2), hh2, T(-1));
    Ah = fma(T(-2), eh, Ah);
    Ah = fma(p, fma(T(2), e32, T(-2.0 / 3.0)), Ah);
    Ah = fma(p2, fma(T(-10.0 / 3.0), e32, T(2.0 / 3.0)), Ah);
    T Bh = fma(T(-6), hh2, T(-1));
    Bh = fma(T(6), eh, Bh);
    Bh = fma(p, fma(T(-10), e32, T(2)), Bh);
    Bh = fma(p2, fma(T(70.0 / 3.0), e32, T(-10.0 / 3.0)), Bh);
    T Ch = hh * fma(T(-12), e32, T(2));
    Ch = fma(T(12) * eh, hh, Ch);
    Ch = fma(e3, fma(p, fma(T(20), e32, T(-4)), p2 * fma(T(-140.0 / 3.0), e32, T(40.0 / 3.0))),
             Ch);
    const T Dh = fma(T(-20.0 / 3.0), p2 * e3, T(2) * hh);
    T Eh = p2 * fma(T(20), e32, T(-8.0 / 3.0));
    Eh = fma(T(-4), p * e32, Eh);
    Eh = fma(T(-4), hh2, Eh);
    // v = Ri [A^ l + e (B^ s + C^ lz) + z (D^ s + E^ lz)],  s = e.l,  e = R Ri
    const T s = Ri * fma(dx, lx, fma(dy, ly, Rz * lz));
    const T t1 = fma(Bh, s, Ch * lz) * Ri2;
    const T t2 = fma(Dh, s, Eh * lz) * Ri;
    const T AR = Ah * Ri;
    ax = fma(AR, lx, fma(t1, dx, ax));
    ay = fma(AR, ly, fma(t1, dy, ay));
    az = fma(AR, lz, fma(t1, Rz, az)) + t2;
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
    const double rinv = r2 > 0.0 ? rsq_f64(r2) : 0.0;
    const double Rz = zt + zs;
    const double Ri = wall ? rsq_f64(fma(Rz, Rz, dxy2)) : 0.0;
    for (int col = 0; col < 3; ++col) {
        const double lx = col == 0, ly = col == 1, lz = col == 2;
        double ax = 0.0, ay = 0.0, az = 0.0;
        rpy_free<double>(dx, dy, dz, r2, rinv, lx, ly, lz, c, ax, ay, az);
        if (wall) rpy_image<double>(dx, dy, Rz, zs, Ri, lx, ly, lz, c, ax, ay, az);
        B[col] = ax;
        B[3 + col] = ay;
        B[6 + col] = az;
    }
}

}  // namespace arb
