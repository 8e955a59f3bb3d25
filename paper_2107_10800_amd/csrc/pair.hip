// Blob-blob RPY mobility product u = M lambda on gfx950 (Sec. 2.3, Eq. RPY).
//
// Pair tensor, in units of 1/(8 pi eta), for r = r_i - r_j (target minus source):
//   unbounded (Rotne-Prager / Wajnryb et al.):
//     r >  2a: c1 I + c2 r r^T,  c1 = (1 + 2a^2/(3 r^2))/r,  c2 = (1 - 2a^2/r^2)/r^3
//     r <= 2a: c1 = 4/(3a) - 3r/(8a^2),  c2 = 1/(8 a^2 r)  (c2 r r^T -> 0 at r = 0)
//   no-slip wall at z = 0 (Swan & Brady): add the Faxen-regularised image of
//   Blake's solution.  With R = (x - y*) for the source image y* = (y1,y2,-y3),
//   e = R/|R|, h = source height, p = a^2/|R|^2, hh = h/|R|, the image is
//     I = (1/|R|) [A^ delta + B^ e e^T + C^ e z^T + D^ z e^T + E^ z z^T]
//   with the scalar polynomials (z = unit wall normal, e3 = e.z)
//     A^ = -1 + 2hh^2 - 2 e3 hh + p(2e3^2 - 2/3) + p^2(2/3 - 10e3^2/3)
//     B^ = -1 - 6hh^2 + 6 e3 hh + p(2 - 10e3^2) + p^2(70e3^2/3 - 10/3)
//     C^ = hh(2 - 12e3^2) + 12 e3 hh^2 + e3 [p(20e3^2 - 4) + p^2(40/3 - 140e3^2/3)]
//     D^ = 2hh - (20/3) p^2 e3
//     E^ = -4hh^2 - 4 p e3^2 + p^2(20e3^2 - 8/3)
//   obtained by applying (1 + a^2/6 lap_x)(1 + a^2/6 lap_y) to Blake's image
//   system and collecting terms (the same expression at x = y is the blob's
//   wall-corrected self mobility).
//
// Launch: grid (ceil(N/256) target blocks) x (source slices).  Each thread owns
// one target; the block streams its slice's sources through LDS in tiles of
// 256 (x,y,z + lambda), all lanes reading the same LDS word (broadcast).  Each
// slice writes its partial sums; pair_reduce adds slices in a fixed order, so
// results are deterministic.  FP32C: positions (in units of a) are split hi +
// lo floats so that differences keep ~double accuracy; sums are float over
// runs of 32 sources and double across runs.
#include "rpy_device.h"

namespace arb {

// p64: positions (w = 2 z); hi + lo: positions / a split into two floats, with
// hi.w = 2 hi.z and lo.w = -(2 hi.z)^2, the source-height terms of the wall image.
// box (may be null): per tile of 64 consecutive blobs (one wavefront here),
// box[2t] = (min x, min y, min z, max |coordinate|) and box[2t+1] = (max x,
// max y, max z, 0) of the hi positions, for the symmetric kernel's far test.
// perm (may be null): entry i holds blob perm[i] (the pair kernels' blob order)
__global__ void prep_positions_kernel(int N, const double *__restrict__ pos, double inv_a,
                                      double sx, double sy, double4 *__restrict__ p64,
                                      float4 *__restrict__ hi, float4 *__restrict__ lo,
                                      float4 *__restrict__ box, const int *__restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < N;
    float xh = 0.f, yh = 0.f, zh = 0.f;
    if (ok) {
        const int b = perm ? perm[i] : i;
        const double px = pos[3 * b] - sx, py = pos[3 * b + 1] - sy, pz = pos[3 * b + 2];
        p64[i] = make_double4(px, py, pz, 2.0 * pz);
        const double x = px * inv_a, y = py * inv_a, z = pz * inv_a;
        xh = (float)x;
        yh = (float)y;
        zh = (float)z;
        const float h2 = 2.f * zh;
        hi[i] = make_float4(xh, yh, zh, h2);
        lo[i] = make_float4((float)(x - (double)xh), (float)(y - (double)yh),
                            (float)(z - (double)zh), -(h2 * h2));
    }
    if (!box) return;
    const float inf = __int_as_float(0x7f800000);
    float l0 = ok ? xh : inf, l1 = ok ? yh : inf, l2 = ok ? zh : inf;
    float h0 = ok ? xh : -inf, h1 = ok ? yh : -inf, hz = ok ? zh : -inf;
    float mx = ok ? fmaxf(fabsf(xh), fmaxf(fabsf(yh), fabsf(zh))) : 0.f;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        l0 = fminf(l0, __shfl_xor(l0, off));
        l1 = fminf(l1, __shfl_xor(l1, off));
        l2 = fminf(l2, __shfl_xor(l2, off));
        h0 = fmaxf(h0, __shfl_xor(h0, off));
        h1 = fmaxf(h1, __shfl_xor(h1, off));
        hz = fmaxf(hz, __shfl_xor(hz, off));
        mx = fmaxf(mx, __shfl_xor(mx, off));
    }
    const int t = i / kWave;
    if ((i % kWave) == 0 && t * kWave < N) {
        box[2 * t] = make_float4(l0, l1, l2, mx);
        box[2 * t + 1] = make_float4(h0, h1, hz, 0.f);
    }
}

constexpr int kRun = 32;  // sources per float partial sum in the FP32C kernel

template <bool WALL>
__global__ __launch_bounds__(kTile) void pair_f32c_kernel(
    int N, const float4 *__restrict__ hi, const float4 *__restrict__ lo,
    const double *__restrict__ lam, const int *__restrict__ perm, int tiles_per_slice,
    double *__restrict__ partial) {
    constexpr CoefF c = kUnitCoefF;
    __shared__ float4 s_hi[kTile], s_lo[kTile], s_lam[kTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kTile + tid;
    const int ic = i < N ? i : N - 1;
    const float4 th = hi[ic], tl = lo[ic];
    const float zi = th.z + tl.z;
    const TargetZ<float> zsc = target_z(zi);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    const int ntiles = (N + kTile - 1) / kTile;
    const int t0 = blockIdx.y * tiles_per_slice;
    const int t1 = min(t0 + tiles_per_slice, ntiles);
    for (int t = t0; t < t1; ++t) {
        const int j = t * kTile + tid;
        __syncthreads();
        if (j < N) {
            const size_t b = 3 * (size_t)(perm ? perm[j] : j);
            s_hi[tid] = hi[j];
            s_lo[tid] = lo[j];
            s_lam[tid] = make_float4((float)lam[b], (float)lam[b + 1], (float)lam[b + 2], 0.f);
        }
        __syncthreads();
        const int cnt = min(kTile, N - t * kTile);
        // float sums over runs of kRun sources, promoted to double after each run
        for (int k0 = 0; k0 < cnt; k0 += kRun) {
            const int k1 = min(k0 + kRun, cnt);
            float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 2
            for (int k = k0; k < k1; ++k) {
                const float4 sh = s_hi[k], sl = s_lo[k], L = s_lam[k];
                const float dx = (th.x - sh.x) + (tl.x - sl.x);
                const float dy = (th.y - sh.y) + (tl.y - sl.y);
                const float dz = (th.z - sh.z) + (tl.z - sl.z);
                const float dxy2 = fmaf(dx, dx, dy * dy);
                const float r2 = fmaf(dz, dz, dxy2);
                const float rinv = rsq_f32(r2);
                if (WALL) {
                    const float Rz = zi + sh.z;
                    const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
                    const PairCoef<float> w =
                        wall_pair_coef<float>(r2, rinv, dxy2, zsc, sh.z, sh.w, sl.w, Rz, Ri, c);
                    wall_pair_apply<float>(w, w.c, w.d, dx, dy, dz, Rz, L.x, L.y, L.z, ax, ay, az);
                } else {
                    rpy_free<float>(dx, dy, dz, r2, rinv, L.x, L.y, L.z, c, ax, ay, az);
                }
            }
            ux += (double)ax;
            uy += (double)ay;
            uz += (double)az;
        }
    }
    if (i < N) {
        const size_t base = (size_t)blockIdx.y * 3 * N + i;
        partial[base] = ux;
        partial[base + N] = uy;
        partial[base + 2 * (size_t)N] = uz;
    }
}

template <bool WALL>
__global__ __launch_bounds__(kTile) void pair_f64_kernel(int N, const double4 *__restrict__ p64,
                                                         const double *__restrict__ lam,
                                                         const int *__restrict__ perm,
                                                         int tiles_per_slice, CoefD c,
                                                         double *__restrict__ partial) {
    __shared__ double4 s_p[kTile];
    __shared__ double s_l[3 * kTile];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * kTile + tid;
    const int ic = i < N ? i : N - 1;
    const double4 ti = p64[ic];
    const TargetZ<double> zsc = target_z(ti.z);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    const int ntiles = (N + kTile - 1) / kTile;
    const int t0 = blockIdx.y * tiles_per_slice;
    const int t1 = min(t0 + tiles_per_slice, ntiles);
    for (int t = t0; t < t1; ++t) {
        const int j = t * kTile + tid;
        __syncthreads();
        if (j < N) {
            const size_t b = 3 * (size_t)(perm ? perm[j] : j);
            s_p[tid] = p64[j];
            s_l[3 * tid] = lam[b];
            s_l[3 * tid + 1] = lam[b + 1];
            s_l[3 * tid + 2] = lam[b + 2];
        }
        __syncthreads();
        const int cnt = min(kTile, N - t * kTile);
        for (int k = 0; k < cnt; ++k) {
            const double4 sj = s_p[k];
            const double lx = s_l[3 * k], ly = s_l[3 * k + 1], lz = s_l[3 * k + 2];
            const double dx = ti.x - sj.x, dy = ti.y - sj.y, dz = ti.z - sj.z;
            const double dxy2 = fma(dx, dx, dy * dy);
            const double r2 = fma(dz, dz, dxy2);
            const double rinv = rsq_f64(r2);
            if (WALL) {
                const double Rz = ti.z + sj.z;
                const double Ri = rsq_f64(fma(Rz, Rz, dxy2));
                const PairCoef<double> w =
                    wall_pair_coef<double>(r2, rinv, dxy2, zsc, sj.z, sj.w, -(sj.w * sj.w), Rz, Ri, c);
                wall_pair_apply<double>(w, w.c, w.d, dx, dy, dz, Rz, lx, ly, lz, ux, uy, uz);
            } else {
                rpy_free<double>(dx, dy, dz, r2, rinv, lx, ly, lz, c, ux, uy, uz);
            }
        }
    }
    if (i < N) {
        const size_t base = (size_t)blockIdx.y * 3 * N + i;
        partial[base] = ux;
        partial[base + N] = uy;
        partial[base + 2 * (size_t)N] = uz;
    }
}

// partial in the pair kernels' order (entry k = blob perm[k]); out in blob order
__global__ void pair_reduce_kernel(int N, int slices, const double *__restrict__ partial,
                                   double scale, double *__restrict__ out,
                                   const double *__restrict__ U, const int *__restrict__ bob,
                                   const double *__restrict__ dvec, const int *__restrict__ perm) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int i = perm ? perm[k] : k;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int s = 0; s < slices; ++s) {
        const size_t base = (size_t)s * 3 * N + k;
        s0 += partial[base];
        s1 += partial[base + N];
        s2 += partial[base + 2 * (size_t)N];
    }
    s0 *= scale;
    s1 *= scale;
    s2 *= scale;
    if (U) {
        // subtract (K U)_i = u_p + w_p x d_i  (Eq. no-slip)
        const double *Up = U + 6 * (size_t)bob[i];
        const double d0 = dvec[3 * i], d1 = dvec[3 * i + 1], d2 = dvec[3 * i + 2];
        s0 -= Up[0] + (Up[4] * d2 - Up[5] * d1);
        s1 -= Up[1] + (Up[5] * d0 - Up[3] * d2);
        s2 -= Up[2] + (Up[3] * d1 - Up[4] * d0);
    }
    out[3 * i] = s0;
    out[3 * i + 1] = s1;
    out[3 * i + 2] = s2;
}

__global__ void wall_check_kernel(int N, const double4 *__restrict__ p64, double a,
                                  int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && !(p64[i].z > a)) atomicOr(flag, 1);
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void prep_positions(hipStream_t s, int N, const double *pos_aos, double a, double4 *p64,
                    float4 *hi, float4 *lo, float4 *box, const int *perm, double sx, double sy) {
    if (N <= 0) return;
    prep_positions_kernel<<<nblk(N, 256), 256, 0, s>>>(N, pos_aos, 1.0 / a, sx, sy, p64, hi, lo,
                                                       box, perm);
}

int heuristic_slices(int N) {
    const int ntiles = (N + kTile - 1) / kTile;
    int s = 1;
    while ((int64_t)ntiles * s * 2 <= 2048 && s * 2 <= ntiles) s *= 2;
    return s;
}

// Small systems (N <= kSmallPairN, e.g. a 20-rod filament of 80 blobs): one
// 64-lane workgroup per (64 targets, run of kSmallRun sources), sources read
// straight from memory, so that a product of a few thousand pairs spreads over
// N/64 x N/16 wavefronts instead of one workgroup; partial[run][c][i], reduced in
// run order by pair_reduce (deterministic).
template <bool WALL>
__global__ __launch_bounds__(64) void pair_small_f64_kernel(int N, const double4 *__restrict__ p64,
                                                            const double *__restrict__ lam,
                                                            const int *__restrict__ perm, CoefD c,
                                                            double *__restrict__ partial) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int ic = i < N ? i : N - 1;
    const double4 ti = p64[ic];
    const TargetZ<double> zsc = target_z(ti.z);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    const int j0 = blockIdx.y * kSmallRun, j1 = min(j0 + kSmallRun, N);
    for (int j = j0; j < j1; ++j) {
        const double4 sj = p64[j];
        const size_t b = 3 * (size_t)(perm ? perm[j] : j);
        const double lx = lam[b], ly = lam[b + 1], lz = lam[b + 2];
        const double dx = ti.x - sj.x, dy = ti.y - sj.y, dz = ti.z - sj.z;
        const double dxy2 = fma(dx, dx, dy * dy);
        const double r2 = fma(dz, dz, dxy2);
        const double rinv = rsq_f64(r2);
        if (WALL) {
            const double Rz = ti.z + sj.z;
            const double Ri = rsq_f64(fma(Rz, Rz, dxy2));
            const PairCoef<double> w =
                wall_pair_coef<double>(r2, rinv, dxy2, zsc, sj.z, sj.w, -(sj.w * sj.w), Rz, Ri, c);
            wall_pair_apply<double>(w, w.c, w.d, dx, dy, dz, Rz, lx, ly, lz, ux, uy, uz);
        } else {
            rpy_free<double>(dx, dy, dz, r2, rinv, lx, ly, lz, c, ux, uy, uz);
        }
    }
    if (i < N) {
        const size_t base = (size_t)blockIdx.y * 3 * N + i;
        partial[base] = ux;
        partial[base + N] = uy;
        partial[base + 2 * (size_t)N] = uz;
    }
}

template <bool WALL>
__global__ __launch_bounds__(64) void pair_small_f32c_kernel(int N, const float4 *__restrict__ hi,
                                                             const float4 *__restrict__ lo,
                                                             const double *__restrict__ lam,
                                                             const int *__restrict__ perm,
                                                             double *__restrict__ partial) {
    constexpr CoefF c = kUnitCoefF;
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int ic = i < N ? i : N - 1;
    const float4 th = hi[ic], tl = lo[ic];
    const float zi = th.z + tl.z;
    const TargetZ<float> zsc = target_z(zi);
    float ax = 0.f, ay = 0.f, az = 0.f;  // one float run of at most kSmallRun sources
    const int j0 = blockIdx.y * kSmallRun, j1 = min(j0 + kSmallRun, N);
    for (int j = j0; j < j1; ++j) {
        const float4 sh = hi[j], sl = lo[j];
        const size_t b = 3 * (size_t)(perm ? perm[j] : j);
        const float Lx = (float)lam[b], Ly = (float)lam[b + 1], Lz = (float)lam[b + 2];
        const float dx = (th.x - sh.x) + (tl.x - sl.x);
        const float dy = (th.y - sh.y) + (tl.y - sl.y);
        const float dz = (th.z - sh.z) + (tl.z - sl.z);
        const float dxy2 = fmaf(dx, dx, dy * dy);
        const float r2 = fmaf(dz, dz, dxy2);
        const float rinv = rsq_f32(r2);
        if (WALL) {
            const float Rz = zi + sh.z;
            const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
            const PairCoef<float> w =
                wall_pair_coef<float>(r2, rinv, dxy2, zsc, sh.z, sh.w, sl.w, Rz, Ri, c);
            wall_pair_apply<float>(w, w.c, w.d, dx, dy, dz, Rz, Lx, Ly, Lz, ax, ay, az);
        } else {
            rpy_free<float>(dx, dy, dz, r2, rinv, Lx, Ly, Lz, c, ax, ay, az);
        }
    }
    if (i < N) {
        const size_t base = (size_t)blockIdx.y * 3 * N + i;
        partial[base] = (double)ax;
        partial[base + N] = (double)ay;
        partial[base + 2 * (size_t)N] = (double)az;
    }
}

int pair_partial_small(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
                       const float4 *hi, const float4 *lo, const double *lam, const int *perm,
                       double a, double *partial) {
    if (N <= 0) return 0;
    const int runs = (N + kSmallRun - 1) / kSmallRun;
    dim3 grid((N + 63) / 64, runs);
    if (precision == ARB_FP32C) {
        if (wall)
            pair_small_f32c_kernel<true><<<grid, 64, 0, s>>>(N, hi, lo, lam, perm, partial);
        else
            pair_small_f32c_kernel<false><<<grid, 64, 0, s>>>(N, hi, lo, lam, perm, partial);
    } else {
        const CoefD c = make_coef<CoefD, double>(a);
        if (wall)
            pair_small_f64_kernel<true><<<grid, 64, 0, s>>>(N, p64, lam, perm, c, partial);
        else
            pair_small_f64_kernel<false><<<grid, 64, 0, s>>>(N, p64, lam, perm, c, partial);
    }
    return runs;
}

int pair_partial(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
                  const float4 *hi, const float4 *lo, const double *lam, const int *perm, double a,
                  int slices, double *partial) {
    if (N <= 0) return 0;
    const int ntiles = (N + kTile - 1) / kTile;
    if (slices > ntiles) slices = ntiles;
    const int tps = (ntiles + slices - 1) / slices;
    dim3 grid(ntiles, slices);
    if (precision == ARB_FP32C) {
        if (wall)
            pair_f32c_kernel<true><<<grid, kTile, 0, s>>>(N, hi, lo, lam, perm, tps, partial);
        else
            pair_f32c_kernel<false><<<grid, kTile, 0, s>>>(N, hi, lo, lam, perm, tps, partial);
    } else {
        const CoefD c = make_coef<CoefD, double>(a);
        if (wall)
            pair_f64_kernel<true><<<grid, kTile, 0, s>>>(N, p64, lam, perm, tps, c, partial);
        else
            pair_f64_kernel<false><<<grid, kTile, 0, s>>>(N, p64, lam, perm, tps, c, partial);
    }
    return slices;
}

void pair_reduce(hipStream_t s, int N, int slices, const double *partial, double scale,
                 double *out, const double *U, const int *body_of_blob, const double *dvec,
                 const int *perm) {
    if (N <= 0) return;
    pair_reduce_kernel<<<nblk(N, 256), 256, 0, s>>>(N, slices, partial, scale, out, U,
                                                      body_of_blob, dvec, perm);
}

int pair_wall_violation(hipStream_t s, int N, const double4 *p64, double a, int *flag_dev,
                        int *flag_host) {
    if (N <= 0) return 0;
    (void)hipMemsetAsync(flag_dev, 0, sizeof(int), s);
    wall_check_kernel<<<nblk(N, 256), 256, 0, s>>>(N, p64, a, flag_dev);
    (void)hipMemcpyAsync(flag_host, flag_dev, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    return *flag_host;
}

}  // namespace arb
