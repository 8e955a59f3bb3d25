// Symmetric blob-pair product u = M lambda (Sec. 2.3, Eq. RPY), FP32 and FP64.
//
// The pair tensor obeys M(x_j, x_i) = M(x_i, x_j)^T (reciprocity of the RPY and
// wall-corrected RPY tensors), so each unordered pair is evaluated once and
// applied to both blobs: u_i += M_ij lambda_j and u_j += M_ij^T lambda_i.  With
// the coefficients of rpy_device.h the transpose only swaps two scalars.
//
// Work decomposition: tiles of 64 blobs; an "I-block" is 4 consecutive tiles
// (256 targets, one per thread of a 256-thread block).  One launch runs a work
// list of two kinds of items:
//   * off-diagonal (b, J0, nJ, 0): I-block b against source tiles J0..J0+nJ-1
//     with J0 >= 4b+4, so every tile pair (I < J) across blocks is visited once.
//     Each wavefront keeps its 64 targets in registers; the source tile is
//     staged in LDS; at step s lane l meets source (l + s) mod 64 and its
//     source-side accumulator moves one lane down after each step (a wave
//     shuffle), so after 64 steps lane l holds source l's sum.  The 4
//     wavefronts' source sums are added in LDS and then to u in FP64 (device
//     atomics);
//   * diagonal (b, 4b, nJ, 1): all ordered pairs among I-block b's own tiles,
//     target side only (the self pair included).
// FP32 (positions in units of a, split hi + lo): float sums over one source
// tile, promoted to FP64 per tile.  FP64: the same work list with double positions and sums.
// Target sums are promoted to FP64 after each source tile and added to u at the
// end of the item.  u is cleared first; FP64 addition order of the atomics
// varies between runs (results reproducible to FP64 rounding).  Rows beyond N
// are padded with far-away zero-force blobs.
#include <algorithm>
#include <vector>

#include "rpy_device.h"

namespace arb {

// accumulate the free-space tensor both ways: f += M lj, a += M li (NEAR as in
// wall_pair_coef)
template <class T, class C, bool NEAR = true>
__device__ __forceinline__ void sym_free(T dx, T dy, T dz, T r2, T rinv, T lix, T liy, T liz,
                                         T ljx, T ljy, T ljz, const C &c, T &fx, T &fy, T &fz,
                                         T &ax, T &ay, T &az) {
    const T rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
    T c1 = fma(c.k1, rinv3, rinv);
    T c2 = fma(-c.k2, rinv3 * rinv2, rinv3);
    if (NEAR) {
        ARB_IF_ANY_OVERLAP(r2 <= c.four_a2)
        if (r2 <= c.four_a2) {
            const T rv = r2 > T(0) ? rinv : T(0);
            c1 = fma(-c.n2, r2 * rv, c.n1);
            c2 = rv * c.n3;
        }
        ARB_END_IF_ANY
    }
    const T tj = c2 * fma(dx, ljx, fma(dy, ljy, dz * ljz));
    const T ti = c2 * fma(dx, lix, fma(dy, liy, dz * liz));
    fx = fma(c1, ljx, fma(tj, dx, fx));
    fy = fma(c1, ljy, fma(tj, dy, fy));
    fz = fma(c1, ljz, fma(tj, dz, fz));
    ax = fma(c1, lix, fma(ti, dx, ax));
    ay = fma(c1, liy, fma(ti, dy, ay));
    az = fma(c1, liz, fma(ti, dz, az));
}

// v of lane (l + 1) mod 64 for lane l: DPP wave_rol:1 (a VALU move across the
// whole wavefront)
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xF, 0xF,
                                                      false));
}

__device__ __forceinline__ double from_next_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x134, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x134, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct Blob32 {
    float4 hi, lo, lam;
};

// entry i (blob perm[i], or blob i without perm), or a far-away zero-force blob
// beyond N
__device__ __forceinline__ Blob32 load_blob(int i, int N, const float4 *__restrict__ hi,
                                            const float4 *__restrict__ lo,
                                            const double *__restrict__ lam,
                                            const int *__restrict__ perm) {
    Blob32 b;
    if (i < N) {
        const size_t l = 3 * (size_t)(perm ? perm[i] : i);
        b.hi = hi[i];
        b.lo = lo[i];
        b.lam = make_float4((float)lam[l], (float)lam[l + 1], (float)lam[l + 2], 0.f);
    } else {
        b.hi = make_float4(1e6f, 1e6f, 10.f, 20.f);
        b.lo = make_float4(0.f, 0.f, 0.f, -400.f);
        b.lam = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return b;
}

__global__ void zero_kernel(size_t n, double *__restrict__ u) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = 0.0;
}

// far test of a target tile against a source tile (units of a): the gap between
// their boxes is at least kFarMin and at least kFarRel times the sum of their
// largest |coordinates|, so that the hi parts alone give every difference to a
// relative 2^-20 (hi rounding <= |x| 2^-24 per coordinate, sqrt(3) 2^-23 (|x_i| +
// |x_j|) / r <= 2^-20 for r >= 0.11 (|x_i| + |x_j|)), and every pair is far from
// overlapping (r > 2a)
constexpr float kFarMin = 8.f;
constexpr float kFarRel = 0.11f;

// one source tile (staged twice over in LDS) against this lane's target, both ways;
// NEAR: hi + lo differences and the overlap branch; else hi differences only
template <bool WALL, bool NEAR>
__device__ __forceinline__ void sym_tile_loop(const Blob32 &t, float zi, const TargetZ<float> &zsc,
                                              int lane, int src, const float4 *s_hi,
                                              const float4 *s_lo, const float4 *s_lam, float &fx,
                                              float &fy, float &fz, float &ax, float &ay,
                                              float &az) {
    constexpr CoefF c = kUnitCoefF;
#pragma unroll 2
    for (int st = 0; st < 64; ++st) {
        const int k = lane + st;
        const float4 sh = s_hi[k], L = s_lam[k];
        float dx, dy, dz, mh22;
        if (NEAR) {
            const float4 sl = s_lo[k];
            dx = (t.hi.x - sh.x) + (t.lo.x - sl.x);
            dy = (t.hi.y - sh.y) + (t.lo.y - sl.y);
            dz = (t.hi.z - sh.z) + (t.lo.z - sl.z);
            mh22 = sl.w;
        } else {
            dx = t.hi.x - sh.x;
            dy = t.hi.y - sh.y;
            dz = t.hi.z - sh.z;
            mh22 = s_lo[k].w;
        }
        const float dxy2 = fmaf(dx, dx, dy * dy);
        const float r2 = fmaf(dz, dz, dxy2);
        const float rinv = rsq_f32(r2);
        if (WALL) {
            const float Rz = zi + sh.z;
            const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
            const PairCoef<float> q = wall_pair_coef<float, CoefF, NEAR>(r2, rinv, dxy2, zsc, sh.z,
                                                                         sh.w, mh22, Rz, Ri, c);
            wall_pair_apply<float>(q, q.c, q.d, dx, dy, dz, Rz, L.x, L.y, L.z, fx, fy, fz);
            wall_pair_apply<float>(q, q.d, q.c, dx, dy, dz, Rz, t.lam.x, t.lam.y, t.lam.z, ax, ay,
                                   az);
        } else {
            sym_free<float, CoefF, NEAR>(dx, dy, dz, r2, rinv, t.lam.x, t.lam.y, t.lam.z, L.x, L.y,
                                         L.z, c, fx, fy, fz, ax, ay, az);
        }
        // the source-side sums follow their sources: lane l takes lane l+1's.
        // The free-space loop has VALU to spare and waits on the LDS, so it
        // rotates with a whole-wave DPP move; the wall loop is VALU-bound and
        // uses the LDS crossbar.
        if (WALL) {
            ax = __shfl(ax, src);
            ay = __shfl(ay, src);
            az = __shfl(az, src);
        } else {
            ax = from_next_lane(ax);
            ay = from_next_lane(ay);
            az = from_next_lane(az);
        }
    }
}

template <bool WALL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6)))
void pair_sym_f32c_kernel(int N, const float4 *__restrict__ hi,
                                                            const float4 *__restrict__ lo,
                                                            const float4 *__restrict__ box,
                                                            const double *__restrict__ lam,
                                                            const int *__restrict__ perm,
                                                            const int4 *__restrict__ work,
                                                            double *__restrict__ u) {
    constexpr CoefF c = kUnitCoefF;
    // the source tile twice over, so the rotation reads lane + step without wrapping
    __shared__ float4 s_hi[128], s_lo[128], s_lam[128];
    __shared__ float comb[4][3][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int4 it = work[blockIdx.x];
    const bool diag = it.w != 0;
    const int i = (4 * it.x + w) * 64 + lane;
    const Blob32 t = load_blob(i, N, hi, lo, lam, perm);
    const float zi = t.hi.z + t.lo.z;
    const TargetZ<float> zsc = target_z(zi);
    const int src = (lane + 1) & 63;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    for (int J = it.y; J < it.y + it.z; ++J) {
        __syncthreads();
        if (tid < 64) {
            const Blob32 s = load_blob(J * 64 + tid, N, hi, lo, lam, perm);
            s_hi[tid] = s_hi[tid + 64] = s.hi;
            s_lo[tid] = s_lo[tid + 64] = s.lo;
            s_lam[tid] = s_lam[tid + 64] = s.lam;
        }
        __syncthreads();
        float fx = 0.f, fy = 0.f, fz = 0.f;
        if (diag) {
#pragma unroll 2
            for (int k = 0; k < 64; ++k) {
                const float4 sh = s_hi[k], sl = s_lo[k], L = s_lam[k];
                const float dx = (t.hi.x - sh.x) + (t.lo.x - sl.x);
                const float dy = (t.hi.y - sh.y) + (t.lo.y - sl.y);
                const float dz = (t.hi.z - sh.z) + (t.lo.z - sl.z);
                const float dxy2 = fmaf(dx, dx, dy * dy);
                const float r2 = fmaf(dz, dz, dxy2);
                const float rinv = rsq_f32(r2);
                if (WALL) {
                    const float Rz = zi + sh.z;
                    const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
                    const PairCoef<float> q =
                        wall_pair_coef<float>(r2, rinv, dxy2, zsc, sh.z, sh.w, sl.w, Rz, Ri, c);
                    wall_pair_apply<float>(q, q.c, q.d, dx, dy, dz, Rz, L.x, L.y, L.z, fx, fy, fz);
                } else {
                    rpy_free<float>(dx, dy, dz, r2, rinv, L.x, L.y, L.z, c, fx, fy, fz);
                }
            }
        } else {
            float ax = 0.f, ay = 0.f, az = 0.f;
            // far: every pair of the two tiles is farther apart than the FP32 hi parts
            // alone resolve to 2^-20 (the lo parts dropped, no overlap possible)
            bool far = false;
            if (box) {
                // this wavefront's target tile and the source tile (read again per
                // source tile: L2-resident, and no registers held across the loop)
                const float4 tl_ = box[2 * (4 * it.x + w)], th = box[2 * (4 * it.x + w) + 1];
                const float4 jl = box[2 * J], jh = box[2 * J + 1];
                const float gx = fmaxf(0.f, fmaxf(jl.x - th.x, tl_.x - jh.x));
                const float gy = fmaxf(0.f, fmaxf(jl.y - th.y, tl_.y - jh.y));
                const float gz = fmaxf(0.f, fmaxf(jl.z - th.z, tl_.z - jh.z));
                const float thr = fmaxf(kFarMin, kFarRel * (tl_.w + jl.w));
                far = fmaf(gx, gx, fmaf(gy, gy, gz * gz)) >= thr * thr;
            }
            if (far)
                sym_tile_loop<WALL, false>(t, zi, zsc, lane, src, s_hi, s_lo, s_lam, fx, fy, fz, ax,
                                           ay, az);
            else
                sym_tile_loop<WALL, true>(t, zi, zsc, lane, src, s_hi, s_lo, s_lam, fx, fy, fz, ax,
                                          ay, az);
            comb[w][0][lane] = ax;
            comb[w][1][lane] = ay;
            comb[w][2][lane] = az;
            __syncthreads();
            if (tid < 192) {
                const int cc = tid >> 6, l = tid & 63;
                const int j = J * 64 + l;
                const float s =
                    (comb[0][cc][l] + comb[1][cc][l]) + (comb[2][cc][l] + comb[3][cc][l]);
                if (j < N) atomicAdd(&u[(size_t)cc * N + j], (double)s);
            }
        }
        ux += (double)fx;
        uy += (double)fy;
        uz += (double)fz;
    }
    if (i < N) {
        atomicAdd(&u[i], ux);
        atomicAdd(&u[(size_t)N + i], uy);
        atomicAdd(&u[2 * (size_t)N + i], uz);
    }
}

// entry i in FP64 (blob perm[i], or blob i), or a far-away zero-force blob beyond N
__device__ __forceinline__ void load_blob64(int i, int N, const double4 *__restrict__ p64,
                                            const double *__restrict__ lam,
                                            const int *__restrict__ perm, double4 &p,
                                            double4 &l) {
    if (i < N) {
        const size_t b = 3 * (size_t)(perm ? perm[i] : i);
        p = p64[i];
        l = make_double4(lam[b], lam[b + 1], lam[b + 2], 0.0);
    } else {
        p = make_double4(1e6, 1e6, 10.0, 20.0);
        l = make_double4(0.0, 0.0, 0.0, 0.0);
    }
}

// the same work list in FP64 (no float runs; sums and the rotation in double)
template <bool WALL>
__global__ __launch_bounds__(256) void pair_sym_f64_kernel(int N, const double4 *__restrict__ p64,
                                                           const double *__restrict__ lam,
                                                           const int *__restrict__ perm,
                                                           const int4 *__restrict__ work,
                                                           CoefD c, double *__restrict__ u) {
    __shared__ double4 s_p[128], s_l[128];  // the source tile twice over
    __shared__ double comb[4][3][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int4 it = work[blockIdx.x];
    const bool diag = it.w != 0;
    const int i = (4 * it.x + w) * 64 + lane;
    double4 tp, tl;
    load_blob64(i, N, p64, lam, perm, tp, tl);
    const TargetZ<double> zsc = target_z(tp.z);
    const int src = (lane + 1) & 63;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int J = it.y; J < it.y + it.z; ++J) {
        __syncthreads();
        if (tid < 64) {
            load_blob64(J * 64 + tid, N, p64, lam, perm, s_p[tid], s_l[tid]);
            s_p[tid + 64] = s_p[tid];
            s_l[tid + 64] = s_l[tid];
        }
        __syncthreads();
        if (diag) {
            for (int k = 0; k < 64; ++k) {
                const double4 sp = s_p[k], L = s_l[k];
                const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
                const double dxy2 = fma(dx, dx, dy * dy);
                const double r2 = fma(dz, dz, dxy2);
                const double rinv = rsq_f64(r2);
                if (WALL) {
                    const double Rz = tp.z + sp.z;
                    const double Ri = rsq_f64(fma(Rz, Rz, dxy2));
                    const PairCoef<double> q =
                        wall_pair_coef<double>(r2, rinv, dxy2, zsc, sp.z, sp.w, -(sp.w * sp.w), Rz,
                                               Ri, c);
                    wall_pair_apply<double>(q, q.c, q.d, dx, dy, dz, Rz, L.x, L.y, L.z, fx, fy, fz);
                } else {
                    rpy_free<double>(dx, dy, dz, r2, rinv, L.x, L.y, L.z, c, fx, fy, fz);
                }
            }
        } else {
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int st = 0; st < 64; ++st) {
                const int k = lane + st;
                const double4 sp = s_p[k], L = s_l[k];
                const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
                const double dxy2 = fma(dx, dx, dy * dy);
                const double r2 = fma(dz, dz, dxy2);
                const double rinv = rsq_f64(r2);
                if (WALL) {
                    const double Rz = tp.z + sp.z;
                    const double Ri = rsq_f64(fma(Rz, Rz, dxy2));
                    const PairCoef<double> q =
                        wall_pair_coef<double>(r2, rinv, dxy2, zsc, sp.z, sp.w, -(sp.w * sp.w), Rz,
                                               Ri, c);
                    wall_pair_apply<double>(q, q.c, q.d, dx, dy, dz, Rz, L.x, L.y, L.z, fx, fy, fz);
                    wall_pair_apply<double>(q, q.d, q.c, dx, dy, dz, Rz, tl.x, tl.y, tl.z, ax, ay,
                                            az);
                } else {
                    sym_free<double>(dx, dy, dz, r2, rinv, tl.x, tl.y, tl.z, L.x, L.y, L.z, c, fx,
                                     fy, fz, ax, ay, az);
                }
                if (WALL) {
                    ax = __shfl(ax, src);
                    ay = __shfl(ay, src);
                    az = __shfl(az, src);
                } else {
                    ax = from_next_lane(ax);
                    ay = from_next_lane(ay);
                    az = from_next_lane(az);
                }
            }
            comb[w][0][lane] = ax;
            comb[w][1][lane] = ay;
            comb[w][2][lane] = az;
            __syncthreads();
            if (tid < 192) {
                const int cc = tid >> 6, l = tid & 63;
                const int j = J * 64 + l;
                const double s =
                    (comb[0][cc][l] + comb[1][cc][l]) + (comb[2][cc][l] + comb[3][cc][l]);
                if (j < N) atomicAdd(&u[(size_t)cc * N + j], s);
            }
        }
    }
    if (i < N) {
        atomicAdd(&u[i], fx);
        atomicAdd(&u[(size_t)N + i], fy);
        atomicAdd(&u[2 * (size_t)N + i], fz);
    }
}

// u = 0 (3N doubles) before the symmetric kernel adds into it
void pair_sym_clear(hipStream_t s, int N, double *u) {
    if (N <= 0) return;
    const size_t n3 = 3 * (size_t)N;
    zero_kernel<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(n3, u);
}

// u (layout [3][N], FP64) += sum over all pairs, unscaled (units 1/(8 pi eta))
void pair_sym(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
              const float4 *hi, const float4 *lo, const float4 *box, const double *lam,
              const int *perm, double a, const int4 *work, int n_work, double *u) {
    if (N <= 0 || n_work <= 0) return;
    if (precision == ARB_FP32C) {
        if (wall)
            pair_sym_f32c_kernel<true><<<n_work, 256, 0, s>>>(N, hi, lo, box, lam, perm, work, u);
        else
            pair_sym_f32c_kernel<false><<<n_work, 256, 0, s>>>(N, hi, lo, box, lam, perm, work, u);
    } else {
        const CoefD c = make_coef<CoefD, double>(a);
        if (wall)
            pair_sym_f64_kernel<true><<<n_work, 256, 0, s>>>(N, p64, lam, perm, work, c, u);
        else
            pair_sym_f64_kernel<false><<<n_work, 256, 0, s>>>(N, p64, lam, perm, work, c, u);
    }
}

// work items: the diagonal item of every I-block, then (b, J0, nJ, 0) covering
// every tile pair I < J across I-blocks in chunks of at most R source tiles;
// ordered by estimated cost, longest first (a diagonal tile costs about 0.6 of
// an off-diagonal one: one direction instead of two)
std::vector<int4> pair_sym_worklist(int N, int R) {
    const int nT = (N + 63) / 64;
    const int nB = (nT + 3) / 4;
    std::vector<int4> items;
    for (int b = 0; b < nB; ++b) items.push_back(make_int4(b, 4 * b, std::min(4, nT - 4 * b), 1));
    for (int b = 0; b < nB; ++b)
        for (int J0 = 4 * b + 4; J0 < nT; J0 += R)
            items.push_back(make_int4(b, J0, std::min(R, nT - J0), 0));
    auto cost = [](const int4 &x) { return x.w ? 0.6 * x.z : (double)x.z; };
    std::stable_sort(items.begin(), items.end(),
                     [&](const int4 &x, const int4 &y) { return cost(x) > cost(y); });
    return items;
}

}  // namespace arb
