// Body mobility of single-blob bodies (Sec. 2.4): the generalised RPY tensor,
// unbounded, applied to the generalised forces (f, tau) of every body,
//     (u_i, w_i) = sum_j N_ij (f_j, tau_j)      (all ordered pairs, i = j included).
// With r = x_i - x_j, r = |r|, in units of 1/(8 pi eta):
//     u_i += c1 f_j + c2 (r . f_j) r + c_r tau_j x r
//     w_i += c_r f_j x r + d1 tau_j + d2 (r . tau_j) r
// translation: c1, c2 of the RPY tensor (as in pair.hip);
// r > 2a : c_r = 1/r^3, d1 = -1/(2 r^3), d2 = 3/(2 r^5);
// r <= 2a: c_r = (1 - 3r/(8a)) / (2a^3),
//          d1 = (1 - 27r/(32a) + 5r^3/(64a^3)) / a^3,
//          d2 = (9/(32 a r) - 3r/(64a^3)) / a^3  (its r r^T term vanishes at r = 0).
// At r = 0 this gives the self mobilities 1/(6 pi eta a), 1/(8 pi eta a^3).
//
// One target body per lane; source tiles of 256 bodies staged in LDS; the
// sources are split into slices (grid y) whose partial sums a second kernel
// adds in slice order (bitwise reproducible), scales and adds to a base vector.
// FP64 in absolute units, or FP32 in units of a (below).
#include "rpy_device.h"

namespace arb {

namespace {

constexpr int kRotTile = 256;

struct RotCoef {
    double k1, k2, n1, n2, n3, four_a2, e1, e2, g0, g1, g3, h1, h3;
};

RotCoef rot_coef(double a) {
    RotCoef c;
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

__global__ __launch_bounds__(kRotTile) void rot_pair_f64_kernel(
    int M, const double4 *__restrict__ p64, const double *__restrict__ x6, int tiles_per_slice,
    RotCoef c, double *__restrict__ partial) {
    __shared__ double4 s_p[kRotTile];
    __shared__ double s_x[6 * kRotTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kRotTile + tid;
    const double4 ti = p64[i < M ? i : M - 1];
    double ux = 0.0, uy = 0.0, uz = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    const int ntiles = (M + kRotTile - 1) / kRotTile;
    const int t0 = blockIdx.y * tiles_per_slice;
    const int t1 = min(t0 + tiles_per_slice, ntiles);
    for (int t = t0; t < t1; ++t) {
        const int j = t * kRotTile + tid;
        __syncthreads();
        if (j < M) {
            s_p[tid] = p64[j];
            for (int k = 0; k < 6; ++k) s_x[6 * tid + k] = x6[6 * (size_t)j + k];
        }
        __syncthreads();
        const int cnt = min(kRotTile, M - t * kRotTile);
        for (int k = 0; k < cnt; ++k) {
            const double4 sj = s_p[k];
            const double *x = s_x + 6 * k;
            const double fx = x[0], fy = x[1], fz = x[2], tx = x[3], ty = x[4], tz = x[5];
            const double dx = ti.x - sj.x, dy = ti.y - sj.y, dz = ti.z - sj.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double rinv = rsq_f64(r2);
            const double rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
            double c1 = fma(c.k1, rinv3, rinv);
            double c2 = fma(-c.k2, rinv3 * rinv2, rinv3);
            double cr = rinv3;
            double d1 = -0.5 * rinv3;
            double d2 = 1.5 * rinv3 * rinv2;
            ARB_IF_ANY_OVERLAP(r2 <= c.four_a2)
            if (r2 <= c.four_a2) {
                const double rv = r2 > 0.0 ? rinv : 0.0;  // rinv is not finite at r = 0
                const double r = r2 * rv;
                c1 = fma(-c.n2, r, c.n1);
                c2 = rv * c.n3;
                cr = fma(-c.e2, r, c.e1);
                d1 = fma(r, fma(c.g3, r * r, -c.g1), c.g0);
                d2 = fma(c.h1, rv, -c.h3 * r);
            }
            ARB_END_IF_ANY
            const double tf = c2 * fma(dx, fx, fma(dy, fy, dz * fz));
            const double tt = d2 * fma(dx, tx, fma(dy, ty, dz * tz));
            // c_r (tau x r) and c_r (f x r) through r scaled by c_r once
            const double ex = cr * dx, ey = cr * dy, ez = cr * dz;
            ux = fma(c1, fx, fma(tf, dx, fma(ty, ez, fma(-tz, ey, ux))));
            uy = fma(c1, fy, fma(tf, dy, fma(tz, ex, fma(-tx, ez, uy))));
            uz = fma(c1, fz, fma(tf, dz, fma(tx, ey, fma(-ty, ex, uz))));
            wx = fma(d1, tx, fma(tt, dx, fma(fy, ez, fma(-fz, ey, wx))));
            wy = fma(d1, ty, fma(tt, dy, fma(fz, ex, fma(-fx, ez, wy))));
            wz = fma(d1, tz, fma(tt, dz, fma(fx, ey, fma(-fy, ex, wz))));
        }
    }
    if (i < M) {
        double *o = partial + (size_t)blockIdx.y * 6 * M + i;
        o[0] = ux;
        o[(size_t)M] = uy;
        o[2 * (size_t)M] = uz;
        o[3 * (size_t)M] = wx;
        o[4 * (size_t)M] = wy;
        o[5 * (size_t)M] = wz;
    }
}

// The same sum in FP32 in units of the blob radius (positions hi + lo = x / a,
// torques scaled by 1/a on loading, literal coefficients for a = 1): then
// u = (1/a) sum and w = (1/a^2) sum, applied by the reduction.  Float sums over
// runs of kRotRun sources are promoted to double after each run.
constexpr int kRotRun = 32;

__global__ __launch_bounds__(kRotTile) void rot_pair_f32c_kernel(
    int M, const float4 *__restrict__ hi, const float4 *__restrict__ lo,
    const double *__restrict__ x6, double inv_a, int tiles_per_slice,
    double *__restrict__ partial) {
    // a = 1: k1 = 2/3, k2 = 2, n1 = 4/3, n2 = 3/8, n3 = 1/8, 4a^2 = 4, e1 = 1/2,
    // e2 = 3/16, g0 = 1, g1 = 27/32, g3 = 5/64, h1 = 9/32, h3 = 3/64
    __shared__ float4 s_hi[kRotTile], s_lo[kRotTile];
    __shared__ float s_x[6 * kRotTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kRotTile + tid;
    const int ic = i < M ? i : M - 1;
    const float4 th = hi[ic], tl = lo[ic];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int ntiles = (M + kRotTile - 1) / kRotTile;
    const int t0 = blockIdx.y * tiles_per_slice;
    const int t1 = min(t0 + tiles_per_slice, ntiles);
    for (int t = t0; t < t1; ++t) {
        const int j = t * kRotTile + tid;
        __syncthreads();
        if (j < M) {
            s_hi[tid] = hi[j];
            s_lo[tid] = lo[j];
            for (int k = 0; k < 6; ++k)
                s_x[6 * tid + k] = (float)(k < 3 ? x6[6 * (size_t)j + k] : x6[6 * (size_t)j + k] * inv_a);
        }
        __syncthreads();
        const int cnt = min(kRotTile, M - t * kRotTile);
        for (int k0 = 0; k0 < cnt; k0 += kRotRun) {
            const int k1 = min(k0 + kRotRun, cnt);
            float ux = 0.f, uy = 0.f, uz = 0.f, wx = 0.f, wy = 0.f, wz = 0.f;
            for (int k = k0; k < k1; ++k) {
                const float4 sh = s_hi[k], sl = s_lo[k];
                const float *x = s_x + 6 * k;
                const float fx = x[0], fy = x[1], fz = x[2], tx = x[3], ty = x[4], tz = x[5];
                const float dx = (th.x - sh.x) + (tl.x - sl.x);
                const float dy = (th.y - sh.y) + (tl.y - sl.y);
                const float dz = (th.z - sh.z) + (tl.z - sl.z);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float rinv = rsq_f32(r2);
                const float rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
                float c1 = fmaf(2.f / 3.f, rinv3, rinv);
                float c2 = fmaf(-2.f, rinv3 * rinv2, rinv3);
                float cr = rinv3;
                float d1 = -0.5f * rinv3;
                float d2 = 1.5f * rinv3 * rinv2;
                ARB_IF_ANY_OVERLAP(r2 <= 4.f)
                if (r2 <= 4.f) {
                    const float rv = r2 > 0.f ? rinv : 0.f;  // rinv is infinite at r = 0
                    const float r = r2 * rv;
                    c1 = fmaf(-3.f / 8.f, r, 4.f / 3.f);
                    c2 = rv * (1.f / 8.f);
                    cr = fmaf(-3.f / 16.f, r, 0.5f);
                    d1 = fmaf(r, fmaf(5.f / 64.f, r * r, -27.f / 32.f), 1.f);
                    d2 = fmaf(9.f / 32.f, rv, -(3.f / 64.f) * r);
                }
                ARB_END_IF_ANY
                const float tf = c2 * fmaf(dx, fx, fmaf(dy, fy, dz * fz));
                const float tt = d2 * fmaf(dx, tx, fmaf(dy, ty, dz * tz));
                const float ex = cr * dx, ey = cr * dy, ez = cr * dz;
                ux = fmaf(c1, fx, fmaf(tf, dx, fmaf(ty, ez, fmaf(-tz, ey, ux))));
                uy = fmaf(c1, fy, fmaf(tf, dy, fmaf(tz, ex, fmaf(-tx, ez, uy))));
                uz = fmaf(c1, fz, fmaf(tf, dz, fmaf(tx, ey, fmaf(-ty, ex, uz))));
                wx = fmaf(d1, tx, fmaf(tt, dx, fmaf(fy, ez, fmaf(-fz, ey, wx))));
                wy = fmaf(d1, ty, fmaf(tt, dy, fmaf(fz, ex, fmaf(-fx, ez, wy))));
                wz = fmaf(d1, tz, fmaf(tt, dz, fmaf(fx, ey, fmaf(-fy, ex, wz))));
            }
            acc[0] += (double)ux;
            acc[1] += (double)uy;
            acc[2] += (double)uz;
            acc[3] += (double)wx;
            acc[4] += (double)wy;
            acc[5] += (double)wz;
        }
    }
    if (i < M) {
        double *o = partial + (size_t)blockIdx.y * 6 * M + i;
        for (int k = 0; k < 6; ++k) o[k * (size_t)M] = acc[k];
    }
}

// out = base + scale_u * sum (u rows) / scale_w * sum (w rows) over slices
// (base may be NULL: zero)
__global__ void rot_reduce_kernel(int M, int slices, const double *__restrict__ partial,
                                  double scale_u, double scale_w,
                                  const double *__restrict__ base, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int sl = 0; sl < slices; ++sl) s += partial[((size_t)sl * 6 + k) * M + i];
        const double b = base ? base[6 * (size_t)i + k] : 0.0;
        out[6 * (size_t)i + k] = fma(k < 3 ? scale_u : scale_w, s, b);
    }
}

}  // namespace

int rot_pair_slices(int M) {
    if (M <= 0) return 1;
    const int ntiles = (M + kRotTile - 1) / kRotTile;
    const int want = (2048 + ntiles - 1) / ntiles;   // about 2,048 workgroups
    return std::max(1, std::min(want, ntiles));
}

void rot_pair_apply(hipStream_t s, int precision, int M, const double4 *p64, const float4 *hi,
                    const float4 *lo, const double *x6, double a, double scale,
                    const double *base, double *partial, double *out) {
    if (M <= 0) return;
    const int ntiles = (M + kRotTile - 1) / kRotTile;
    const int slices = rot_pair_slices(M);
    const int tps = (ntiles + slices - 1) / slices;
    const int used = (ntiles + tps - 1) / tps;
    double su = scale, sw = scale;
    if (precision == ARB_FP32C) {
        rot_pair_f32c_kernel<<<dim3(ntiles, used), kRotTile, 0, s>>>(M, hi, lo, x6, 1.0 / a, tps,
                                                                       partial);
        su = scale / a;
        sw = scale / (a * a);
    } else {
        rot_pair_f64_kernel<<<dim3(ntiles, used), kRotTile, 0, s>>>(M, p64, x6, tps,
                                                                      rot_coef(a), partial);
    }
    rot_reduce_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, used, partial, su, sw, base, out);
}

}  // namespace arb
