// Symmetric blob-pair product for FP32 pair sums (Sec. 2.3, Eq. RPY).
//
// The pair tensor obeys M(x_j, x_i) = M(x_i, x_j)^T (reciprocity of the RPY and
// wall-corrected RPY tensors), so each unordered pair is evaluated once and
// applied to both blobs: u_i += M_ij lambda_j and u_j += M_ij^T lambda_i.  For the
// wall image I = (1/|R|)[A delta + B e e^T + C e z^T + D z e^T + E z z^T] the
// transpose swaps C and D.
//
// Work decomposition: tiles of 64 blobs; an "I-block" is 4 consecutive tiles
// (256 targets, one per thread of a 256-thread block).
//   * pair_diag_f32c_kernel: all ordered pairs inside each I-block (the plain
//     target-parallel loop), written to u (first writer).
//   * pair_sym_f32c_kernel: one work item = (I-block b, source tiles J0..J0+nJ-1)
//     with J0 >= 4b+4, so every tile pair (I < J) is visited exactly once.  Each
//     wavefront keeps its 64 targets in registers; the source tile is staged in
//     LDS; at step s lane l meets source (l + s) mod 64 and its source-side
//     accumulator moves one lane down after each step (a wave shuffle), so after
//     64 steps lane l holds source l's sum.  The 4 wavefronts' source sums are
//     added in LDS and then to u in FP64 (device atomics); target sums are
//     promoted to FP64 after each source tile and added to u at the end.
// Float sums run over at most 64 pairs before promotion to double.  Rows beyond
// N are padded with far-away zero-force blobs.  FP64 addition order of the
// atomics varies between runs (results reproducible to FP64 rounding).
#include <algorithm>
#include <vector>

#include "rpy_device.h"

namespace arb {

// accumulate the free-space tensor both ways: f += M lj, a += M li
__device__ __forceinline__ void sym_free(float dx, float dy, float dz, float r2, float rinv,
                                         float lix, float liy, float liz, float ljx, float ljy,
                                         float ljz, const CoefF &c, float &fx, float &fy,
                                         float &fz, float &ax, float &ay, float &az) {
    const float rinv2 = rinv * rinv;
    float c1 = rinv * fmaf(c.k1, rinv2, 1.f);
    float c2 = rinv * rinv2 * fmaf(-c.k2, rinv2, 1.f);
    if (r2 <= c.four_a2) {
        const float r = r2 * rinv;
        c1 = fmaf(-c.n2, r, c.n1);
        c2 = rinv * c.n3;
    }
    const float tj = c2 * fmaf(dx, ljx, fmaf(dy, ljy, dz * ljz));
    const float ti = c2 * fmaf(dx, lix, fmaf(dy, liy, dz * liz));
    fx = fmaf(c1, ljx, fmaf(tj, dx, fx));
    fy = fmaf(c1, ljy, fmaf(tj, dy, fy));
    fz = fmaf(c1, ljz, fmaf(tj, dz, fz));
    ax = fmaf(c1, lix, fmaf(ti, dx, ax));
    ay = fmaf(c1, liy, fmaf(ti, dy, ay));
    az = fmaf(c1, liz, fmaf(ti, dz, az));
}

// wall image both ways; h = source height zj, Rz = zi + zj
__device__ __forceinline__ void sym_image(float dx, float dy, float Rz, float h, float Ri,
                                          float lix, float liy, float liz, float ljx, float ljy,
                                          float ljz, const CoefF &c, float &fx, float &fy,
                                          float &fz, float &ax, float &ay, float &az) {
    const float e3 = Rz * Ri;
    const float hh = h * Ri;
    const float Ri2 = Ri * Ri;
    const float p = c.a2 * Ri2;
    const float p2 = p * p;
    const float e32 = e3 * e3;
    const float hh2 = hh * hh;
    const float eh = e3 * hh;
    float Ah = fmaf(2.f, hh2, -1.f);
    Ah = fmaf(-2.f, eh, Ah);
    Ah = fmaf(p, fmaf(2.f, e32, -2.f / 3.f), Ah);
    Ah = fmaf(p2, fmaf(-10.f / 3.f, e32, 2.f / 3.f), Ah);
    float Bh = fmaf(-6.f, hh2, -1.f);
    Bh = fmaf(6.f, eh, Bh);
    Bh = fmaf(p, fmaf(-10.f, e32, 2.f), Bh);
    Bh = fmaf(p2, fmaf(70.f / 3.f, e32, -10.f / 3.f), Bh);
    float Ch = hh * fmaf(-12.f, e32, 2.f);
    Ch = fmaf(12.f * eh, hh, Ch);
    Ch = fmaf(e3, fmaf(p, fmaf(20.f, e32, -4.f), p2 * fmaf(-140.f / 3.f, e32, 40.f / 3.f)), Ch);
    const float Dh = fmaf(-20.f / 3.f, p2 * e3, 2.f * hh);
    float Eh = p2 * fmaf(20.f, e32, -8.f / 3.f);
    Eh = fmaf(-4.f, p * e32, Eh);
    Eh = fmaf(-4.f, hh2, Eh);
    const float AR = Ah * Ri;
    // I lj
    const float sj = Ri * fmaf(dx, ljx, fmaf(dy, ljy, Rz * ljz));
    const float t1 = fmaf(Bh, sj, Ch * ljz) * Ri2;
    const float t2 = fmaf(Dh, sj, Eh * ljz) * Ri;
    fx = fmaf(AR, ljx, fmaf(t1, dx, fx));
    fy = fmaf(AR, ljy, fmaf(t1, dy, fy));
    fz = fmaf(AR, ljz, fmaf(t1, Rz, fz)) + t2;
    // I^T li (C and D swap)
    const float si = Ri * fmaf(dx, lix, fmaf(dy, liy, Rz * liz));
    const float q1 = fmaf(Bh, si, Dh * liz) * Ri2;
    const float q2 = fmaf(Ch, si, Eh * liz) * Ri;
    ax = fmaf(AR, lix, fmaf(q1, dx, ax));
    ay = fmaf(AR, liy, fmaf(q1, dy, ay));
    az = fmaf(AR, liz, fmaf(q1, Rz, az)) + q2;
}

struct Blob32 {
    float4 hi, lo, lam;
};

// blob i, or a far-away zero-force blob beyond N
__device__ __forceinline__ Blob32 load_blob(int i, int N, const float4 *__restrict__ hi,
                                            const float4 *__restrict__ lo,
                                            const double *__restrict__ lam) {
    Blob32 b;
    if (i < N) {
        b.hi = hi[i];
        b.lo = lo[i];
        b.lam = make_float4((float)lam[3 * (size_t)i], (float)lam[3 * (size_t)i + 1],
                            (float)lam[3 * (size_t)i + 2], 0.f);
    } else {
        b.hi = make_float4(1e6f, 1e6f, 10.f, 0.f);
        b.lo = make_float4(0.f, 0.f, 0.f, 0.f);
        b.lam = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return b;
}

template <bool WALL>
__global__ __launch_bounds__(256) void pair_diag_f32c_kernel(int N, const float4 *__restrict__ hi,
                                                             const float4 *__restrict__ lo,
                                                             const double *__restrict__ lam,
                                                             CoefF c, double *__restrict__ u) {
    __shared__ float4 s_hi[256], s_lo[256], s_lam[256];
    const int tid = threadIdx.x;
    const int i = blockIdx.x * 256 + tid;
    const Blob32 t = load_blob(i, N, hi, lo, lam);
    s_hi[tid] = t.hi;
    s_lo[tid] = t.lo;
    s_lam[tid] = t.lam;
    __syncthreads();
    const float zi = t.hi.z + t.lo.z;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    for (int k0 = 0; k0 < 256; k0 += 32) {
        float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 2
        for (int k = k0; k < k0 + 32; ++k) {
            const float4 sh = s_hi[k], sl = s_lo[k], L = s_lam[k];
            const float dx = (t.hi.x - sh.x) + (t.lo.x - sl.x);
            const float dy = (t.hi.y - sh.y) + (t.lo.y - sl.y);
            const float dz = (t.hi.z - sh.z) + (t.lo.z - sl.z);
            const float dxy2 = fmaf(dx, dx, dy * dy);
            const float r2 = fmaf(dz, dz, dxy2);
            const float rinv = r2 > 0.f ? rsq_f32(r2) : 0.f;
            rpy_free<float>(dx, dy, dz, r2, rinv, L.x, L.y, L.z, c, ax, ay, az);
            if (WALL) {
                const float Rz = zi + sh.z;
                const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
                rpy_image<float>(dx, dy, Rz, sh.z, Ri, L.x, L.y, L.z, c, ax, ay, az);
            }
        }
        ux += (double)ax;
        uy += (double)ay;
        uz += (double)az;
    }
    if (i < N) {
        u[i] = ux;
        u[(size_t)N + i] = uy;
        u[2 * (size_t)N + i] = uz;
    }
}

template <bool WALL>
__global__ __launch_bounds__(256) void pair_sym_f32c_kernel(int N, const float4 *__restrict__ hi,
                                                            const float4 *__restrict__ lo,
                                                            const double *__restrict__ lam,
                                                            const int4 *__restrict__ work,
                                                            CoefF c, double *__restrict__ u) {
    __shared__ float4 s_hi[64], s_lo[64], s_lam[64];
    __shared__ float comb[4][3][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int4 it = work[blockIdx.x];
    const int i = (4 * it.x + w) * 64 + lane;
    const Blob32 t = load_blob(i, N, hi, lo, lam);
    const float zi = t.hi.z + t.lo.z;
    const int src = (lane + 1) & 63;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    for (int J = it.y; J < it.y + it.z; ++J) {
        __syncthreads();
        if (tid < 64) {
            const Blob32 s = load_blob(J * 64 + tid, N, hi, lo, lam);
            s_hi[tid] = s.hi;
            s_lo[tid] = s.lo;
            s_lam[tid] = s.lam;
        }
        __syncthreads();
        float fx = 0.f, fy = 0.f, fz = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 2
        for (int st = 0; st < 64; ++st) {
            const int k = (lane + st) & 63;
            const float4 sh = s_hi[k], sl = s_lo[k], L = s_lam[k];
            const float dx = (t.hi.x - sh.x) + (t.lo.x - sl.x);
            const float dy = (t.hi.y - sh.y) + (t.lo.y - sl.y);
            const float dz = (t.hi.z - sh.z) + (t.lo.z - sl.z);
            const float dxy2 = fmaf(dx, dx, dy * dy);
            const float r2 = fmaf(dz, dz, dxy2);
            const float rinv = r2 > 0.f ? rsq_f32(r2) : 0.f;
            sym_free(dx, dy, dz, r2, rinv, t.lam.x, t.lam.y, t.lam.z, L.x, L.y, L.z, c, fx, fy, fz,
                     ax, ay, az);
            if (WALL) {
                const float Rz = zi + sh.z;
                const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
                sym_image(dx, dy, Rz, sh.z, Ri, t.lam.x, t.lam.y, t.lam.z, L.x, L.y, L.z, c, fx,
                          fy, fz, ax, ay, az);
            }
            // the source-side sums follow their sources: lane l takes lane l+1's
            ax = __shfl(ax, src);
            ay = __shfl(ay, src);
            az = __shfl(az, src);
        }
        ux += (double)fx;
        uy += (double)fy;
        uz += (double)fz;
        comb[w][0][lane] = ax;
        comb[w][1][lane] = ay;
        comb[w][2][lane] = az;
        __syncthreads();
        if (tid < 192) {
            const int cc = tid >> 6, l = tid & 63;
            const int j = J * 64 + l;
            const float s = (comb[0][cc][l] + comb[1][cc][l]) + (comb[2][cc][l] + comb[3][cc][l]);
            if (j < N) atomicAdd(&u[(size_t)cc * N + j], (double)s);
        }
    }
    if (i < N) {
        atomicAdd(&u[i], ux);
        atomicAdd(&u[(size_t)N + i], uy);
        atomicAdd(&u[2 * (size_t)N + i], uz);
    }
}

// u (layout [3][N], FP64) = sum over all pairs, unscaled (units 1/(8 pi eta))
void pair_sym_f32c(hipStream_t s, bool wall, int N, const float4 *hi, const float4 *lo,
                   const double *lam, double a, const int4 *work, int n_work, double *u) {
    if (N <= 0) return;
    const CoefF c = make_coef<CoefF, float>((float)a);
    const int nblk = (N + 255) / 256;
    if (wall) {
        pair_diag_f32c_kernel<true><<<nblk, 256, 0, s>>>(N, hi, lo, lam, c, u);
        if (n_work > 0) pair_sym_f32c_kernel<true><<<n_work, 256, 0, s>>>(N, hi, lo, lam, work, c, u);
    } else {
        pair_diag_f32c_kernel<false><<<nblk, 256, 0, s>>>(N, hi, lo, lam, c, u);
        if (n_work > 0)
            pair_sym_f32c_kernel<false><<<n_work, 256, 0, s>>>(N, hi, lo, lam, work, c, u);
    }
}

// work items (b, J0, nJ, 0) covering every tile pair I < J across I-blocks,
// chunks of at most R source tiles, longest first
std::vector<int4> pair_sym_worklist(int N, int R) {
    const int nT = (N + 63) / 64;
    const int nB = (nT + 3) / 4;
    std::vector<int4> items;
    for (int b = 0; b < nB; ++b)
        for (int J0 = 4 * b + 4; J0 < nT; J0 += R)
            items.push_back(make_int4(b, J0, std::min(R, nT - J0), 0));
    std::stable_sort(items.begin(), items.end(),
                     [](const int4 &x, const int4 &y) { return x.z > y.z; });
    return items;
}

}  // namespace arb
