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
// N_ji is N_ij with r -> -r: the translation and rotation blocks are even in r,
// the couplings change sign.
//
// Target-parallel form: one target body per lane, source tiles of 256 bodies
// staged in LDS, sources split into slices (grid y) whose partial sums a second
// kernel adds in slice order (bitwise reproducible), scales and adds to a base
// vector.  Symmetric form: the work list of the symmetric wall kernel (each
// 256-body block against itself one way, then 64-body source tiles beyond it
// with both directions from one coefficient evaluation; the source-side sums
// follow their sources around the wavefront by DPP moves), FP64 atomic sums.  FP64 in
// absolute units, or FP32 in units of a (positions hi + lo = x / a, torques
// scaled by 1/a on loading, literal coefficients for a = 1; then u = (1/a) sum
// and w = (1/a^2) sum, applied by the reduction).
#include "rot_device.h"

namespace arb {

namespace {

constexpr int kRotTile = 256;
constexpr int kRotRun = 32;  // sources per float partial sum, target-parallel FP32 kernel

// a += N_ij x_j (target side), b += N_ji x_i (source side: couplings negated)
template <class T>
__device__ __forceinline__ void rot_both(const RotTerms<T> &k, T dx, T dy, T dz, const T *xj,
                                         const T *xi, T *a, T *b) {
    rot_one_way(k, dx, dy, dz, xj[0], xj[1], xj[2], xj[3], xj[4], xj[5], a);
    const T tf = k.c2 * fma(dx, xi[0], fma(dy, xi[1], dz * xi[2]));
    const T tt = k.d2 * fma(dx, xi[3], fma(dy, xi[4], dz * xi[5]));
    const T ex = k.cr * dx, ey = k.cr * dy, ez = k.cr * dz;
    b[0] = fma(k.c1, xi[0], fma(tf, dx, fma(-xi[4], ez, fma(xi[5], ey, b[0]))));
    b[1] = fma(k.c1, xi[1], fma(tf, dy, fma(-xi[5], ex, fma(xi[3], ez, b[1]))));
    b[2] = fma(k.c1, xi[2], fma(tf, dz, fma(-xi[3], ey, fma(xi[4], ex, b[2]))));
    b[3] = fma(k.d1, xi[3], fma(tt, dx, fma(-xi[1], ez, fma(xi[2], ey, b[3]))));
    b[4] = fma(k.d1, xi[4], fma(tt, dy, fma(-xi[2], ex, fma(xi[0], ez, b[4]))));
    b[5] = fma(k.d1, xi[5], fma(tt, dz, fma(-xi[0], ey, fma(xi[1], ex, b[5]))));
}

// ---------------------------------------------------------------- target-parallel form
__global__ __launch_bounds__(kRotTile) void rot_pair_f64_kernel(
    int M, const double4 *__restrict__ p64, const double *__restrict__ x6, int tiles_per_slice,
    RotCoef<double> c, double *__restrict__ partial) {
    __shared__ double4 s_p[kRotTile];
    __shared__ double s_x[6 * kRotTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kRotTile + tid;
    const double4 ti = p64[i < M ? i : M - 1];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
            const double dx = ti.x - sj.x, dy = ti.y - sj.y, dz = ti.z - sj.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const RotTerms<double> kk = rot_terms<double>(r2, rsq_f64(r2), c);
            rot_one_way<double>(kk, dx, dy, dz, x[0], x[1], x[2], x[3], x[4], x[5], acc);
        }
    }
    if (i < M) {
        double *o = partial + (size_t)blockIdx.y * 6 * M + i;
        for (int k = 0; k < 6; ++k) o[k * (size_t)M] = acc[k];
    }
}

// float sums over runs of kRotRun sources, promoted to double after each run
__global__ __launch_bounds__(kRotTile) void rot_pair_f32c_kernel(
    int M, const float4 *__restrict__ hi, const float4 *__restrict__ lo,
    const double *__restrict__ x6, double inv_a, int tiles_per_slice,
    double *__restrict__ partial) {
    constexpr RotCoef<float> c = kUnitRotCoef;
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
                s_x[6 * tid + k] =
                    (float)(k < 3 ? x6[6 * (size_t)j + k] : x6[6 * (size_t)j + k] * inv_a);
        }
        __syncthreads();
        const int cnt = min(kRotTile, M - t * kRotTile);
        for (int k0 = 0; k0 < cnt; k0 += kRotRun) {
            const int k1 = min(k0 + kRotRun, cnt);
            float a[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int k = k0; k < k1; ++k) {
                const float4 sh = s_hi[k], sl = s_lo[k];
                const float *x = s_x + 6 * k;
                const float dx = (th.x - sh.x) + (tl.x - sl.x);
                const float dy = (th.y - sh.y) + (tl.y - sl.y);
                const float dz = (th.z - sh.z) + (tl.z - sl.z);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const RotTerms<float> kk = rot_terms<float>(r2, rsq_f32(r2), c);
                rot_one_way<float>(kk, dx, dy, dz, x[0], x[1], x[2], x[3], x[4], x[5], a);
            }
            for (int k = 0; k < 6; ++k) acc[k] += (double)a[k];
        }
    }
    if (i < M) {
        double *o = partial + (size_t)blockIdx.y * 6 * M + i;
        for (int k = 0; k < 6; ++k) o[k * (size_t)M] = acc[k];
    }
}

// v of lane (l + 1) mod 64 for lane l: DPP wave_rol:1, a VALU move across the
// whole wavefront (the symmetric loops wait on LDS shuffles otherwise)
__device__ __forceinline__ float next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF,
                                                      false));
}
__device__ __forceinline__ double next_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x134, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------- symmetric form
// body j, or a far-away body with zero forces beyond M
__device__ __forceinline__ void load_body64(int j, int M, const double4 *__restrict__ p64,
                                            const double *__restrict__ x6, double4 &p,
                                            double4 &f, double4 &t) {
    if (j < M) {
        p = p64[j];
        const double *x = x6 + 6 * (size_t)j;
        f = make_double4(x[0], x[1], x[2], 0.0);
        t = make_double4(x[3], x[4], x[5], 0.0);
    } else {
        p = make_double4(1e6, 1e6, 1e6, 0.0);
        f = make_double4(0.0, 0.0, 0.0, 0.0);
        t = f;
    }
}

__device__ __forceinline__ void load_body32(int j, int M, const float4 *__restrict__ hi,
                                            const float4 *__restrict__ lo,
                                            const double *__restrict__ x6, double inv_a,
                                            float4 &h, float4 &l, float4 &f, float4 &t) {
    if (j < M) {
        h = hi[j];
        l = lo[j];
        const double *x = x6 + 6 * (size_t)j;
        f = make_float4((float)x[0], (float)x[1], (float)x[2], 0.f);
        t = make_float4((float)(x[3] * inv_a), (float)(x[4] * inv_a), (float)(x[5] * inv_a), 0.f);
    } else {
        h = make_float4(1e6f, 1e6f, 1e6f, 0.f);
        l = make_float4(0.f, 0.f, 0.f, 0.f);
        f = l;
        t = l;
    }
}

// u: [6][M], cleared beforehand
__global__ __launch_bounds__(256) void rot_pair_sym_f64_kernel(int M, const double4 *__restrict__ p64,
                                                               const double *__restrict__ x6,
                                                               const int4 *__restrict__ work,
                                                               RotCoef<double> c,
                                                               double *__restrict__ u) {
    __shared__ double4 s_p[128], s_f[128], s_t[128];  // the source tile twice over
    __shared__ double comb[4][6][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int4 it = work[blockIdx.x];
    const bool diag = it.w != 0;
    const int i = (4 * it.x + w) * 64 + lane;
    double4 tp, tf, tt;
    load_body64(i, M, p64, x6, tp, tf, tt);
    const double xi[6] = {tf.x, tf.y, tf.z, tt.x, tt.y, tt.z};
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int J = it.y; J < it.y + it.z; ++J) {
        __syncthreads();
        if (tid < 64) {
            load_body64(J * 64 + tid, M, p64, x6, s_p[tid], s_f[tid], s_t[tid]);
            s_p[tid + 64] = s_p[tid];
            s_f[tid + 64] = s_f[tid];
            s_t[tid + 64] = s_t[tid];
        }
        __syncthreads();
        if (diag) {
            for (int k = 0; k < 64; ++k) {
                const double4 sp = s_p[k], F = s_f[k], Tq = s_t[k];
                const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const RotTerms<double> kk = rot_terms<double>(r2, rsq_f64(r2), c);
                rot_one_way<double>(kk, dx, dy, dz, F.x, F.y, F.z, Tq.x, Tq.y, Tq.z, a);
            }
        } else {
            double b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int st = 0; st < 64; ++st) {
                const int k = lane + st;
                const double4 sp = s_p[k], F = s_f[k], Tq = s_t[k];
                const double xj[6] = {F.x, F.y, F.z, Tq.x, Tq.y, Tq.z};
                const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const RotTerms<double> kk = rot_terms<double>(r2, rsq_f64(r2), c);
                rot_both<double>(kk, dx, dy, dz, xj, xi, a, b);
                // the source-side sums follow their sources: lane l takes lane l+1's
                for (int q = 0; q < 6; ++q) b[q] = next_lane(b[q]);
            }
            for (int q = 0; q < 6; ++q) comb[w][q][lane] = b[q];
            __syncthreads();
            for (int idx = tid; idx < 6 * 64; idx += 256) {
                const int q = idx >> 6, l = idx & 63;
                const int j = J * 64 + l;
                const double s = (comb[0][q][l] + comb[1][q][l]) + (comb[2][q][l] + comb[3][q][l]);
                if (j < M) atomicAdd(&u[(size_t)q * M + j], s);
            }
        }
    }
    if (i < M)
        for (int q = 0; q < 6; ++q) atomicAdd(&u[(size_t)q * M + i], a[q]);
}

// FP32 in units of a: float sums per 64-body source tile, promoted to double
__global__ __launch_bounds__(256) void rot_pair_sym_f32c_kernel(
    int M, const float4 *__restrict__ hi, const float4 *__restrict__ lo,
    const double *__restrict__ x6, double inv_a, const int4 *__restrict__ work,
    double *__restrict__ u) {
    constexpr RotCoef<float> c = kUnitRotCoef;
    __shared__ float4 s_h[128], s_l[128], s_f[128], s_t[128];
    __shared__ float comb[4][6][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int4 it = work[blockIdx.x];
    const bool diag = it.w != 0;
    const int i = (4 * it.x + w) * 64 + lane;
    float4 th, tl, tf, tt;
    load_body32(i, M, hi, lo, x6, inv_a, th, tl, tf, tt);
    const float xi[6] = {tf.x, tf.y, tf.z, tt.x, tt.y, tt.z};
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int J = it.y; J < it.y + it.z; ++J) {
        __syncthreads();
        if (tid < 64) {
            load_body32(J * 64 + tid, M, hi, lo, x6, inv_a, s_h[tid], s_l[tid], s_f[tid], s_t[tid]);
            s_h[tid + 64] = s_h[tid];
            s_l[tid + 64] = s_l[tid];
            s_f[tid + 64] = s_f[tid];
            s_t[tid + 64] = s_t[tid];
        }
        __syncthreads();
        float a[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (diag) {
            for (int k = 0; k < 64; ++k) {
                const float4 sh = s_h[k], sl = s_l[k], F = s_f[k], Tq = s_t[k];
                const float dx = (th.x - sh.x) + (tl.x - sl.x);
                const float dy = (th.y - sh.y) + (tl.y - sl.y);
                const float dz = (th.z - sh.z) + (tl.z - sl.z);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const RotTerms<float> kk = rot_terms<float>(r2, rsq_f32(r2), c);
                rot_one_way<float>(kk, dx, dy, dz, F.x, F.y, F.z, Tq.x, Tq.y, Tq.z, a);
            }
        } else {
            float b[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int st = 0; st < 64; ++st) {
                const int k = lane + st;
                const float4 sh = s_h[k], sl = s_l[k], F = s_f[k], Tq = s_t[k];
                const float xj[6] = {F.x, F.y, F.z, Tq.x, Tq.y, Tq.z};
                const float dx = (th.x - sh.x) + (tl.x - sl.x);
                const float dy = (th.y - sh.y) + (tl.y - sl.y);
                const float dz = (th.z - sh.z) + (tl.z - sl.z);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const RotTerms<float> kk = rot_terms<float>(r2, rsq_f32(r2), c);
                rot_both<float>(kk, dx, dy, dz, xj, xi, a, b);
                for (int q = 0; q < 6; ++q) b[q] = next_lane(b[q]);
            }
            for (int q = 0; q < 6; ++q) comb[w][q][lane] = b[q];
            __syncthreads();
            for (int idx = tid; idx < 6 * 64; idx += 256) {
                const int q = idx >> 6, l = idx & 63;
                const int j = J * 64 + l;
                const float s = (comb[0][q][l] + comb[1][q][l]) + (comb[2][q][l] + comb[3][q][l]);
                if (j < M) atomicAdd(&u[(size_t)q * M + j], (double)s);
            }
        }
        for (int q = 0; q < 6; ++q) acc[q] += (double)a[q];
    }
    if (i < M)
        for (int q = 0; q < 6; ++q) atomicAdd(&u[(size_t)q * M + i], acc[q]);
}

__global__ void rot_zero_kernel(size_t n, double *__restrict__ u) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) u[k] = 0.0;
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

void rot_reduce(hipStream_t s, int M, const double *partial, double scale_u, double scale_w,
                const double *base, double *out) {
    if (M > 0)
        rot_reduce_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, 1, partial, scale_u, scale_w, base,
                                                          out);
}

int rot_pair_slices(int M) {
    if (M <= 0) return 1;
    const int ntiles = (M + kRotTile - 1) / kRotTile;
    const int want = (2048 + ntiles - 1) / ntiles;   // about 2,048 workgroups
    return std::max(1, std::min(want, ntiles));
}

void rot_pair_apply(hipStream_t s, int precision, int M, const double4 *p64, const float4 *hi,
                    const float4 *lo, const double *x6, double a, double scale,
                    const double *base, double *partial, double *out, const int4 *work,
                    int n_work) {
    if (M <= 0) return;
    const bool f32 = precision == ARB_FP32C;
    const double su = f32 ? scale / a : scale, sw = f32 ? scale / (a * a) : scale;
    int used = 1;
    if (work) {
        const size_t n6 = 6 * (size_t)M;
        rot_zero_kernel<<<(unsigned)((n6 + 255) / 256), 256, 0, s>>>(n6, partial);
        if (n_work > 0) {
            if (f32)
                rot_pair_sym_f32c_kernel<<<n_work, 256, 0, s>>>(M, hi, lo, x6, 1.0 / a, work,
                                                                 partial);
            else
                rot_pair_sym_f64_kernel<<<n_work, 256, 0, s>>>(M, p64, x6, work, rot_coef(a),
                                                                partial);
        }
    } else {
        const int ntiles = (M + kRotTile - 1) / kRotTile;
        const int slices = rot_pair_slices(M);
        const int tps = (ntiles + slices - 1) / slices;
        used = (ntiles + tps - 1) / tps;
        if (f32)
            rot_pair_f32c_kernel<<<dim3(ntiles, used), kRotTile, 0, s>>>(M, hi, lo, x6, 1.0 / a,
                                                                          tps, partial);
        else
            rot_pair_f64_kernel<<<dim3(ntiles, used), kRotTile, 0, s>>>(M, p64, x6, tps,
                                                                          rot_coef(a), partial);
    }
    rot_reduce_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, used, partial, su, sw, base, out);
}

}  // namespace arb
