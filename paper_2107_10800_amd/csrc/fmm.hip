// Fast blob mobility product u = M lambda for large systems (Sec. 2.3; the
// paper names fast summation, Sec. 1 and Sec. 6, as the route past dense sums).
//
// A kernel-independent multipole method (the black-box FMM of Fong and Darve,
// J. Comput. Phys. 228, 2009): the RPY tensor of two well-separated cells is
// replaced by its tensor-product Chebyshev interpolant in both arguments,
//   M(x, y) ~ sum_k sum_m S_k(x) M(t_k, s_m) S_m(y),
// with t, s the n^3 proxy points of the target and source cells.  The pair
// function is the one of the direct sums (unbounded, or with the wall image):
// above the wall nothing else changes, since the image y* of a source is never
// closer to a target than y itself, so a well-separated pair stays
// well-separated for the image term too.
//
// Tree (built on the host once per geometry, in units of length):
//   root cube: origin o = componentwise minimum of the positions, side
//   S = largest extent * (1 + 2^-20) (S = a when all blobs coincide); a blob
//   lies at level l in the cell floor(((x - o) / S) 2^l); cells of one level are
//   adjacent when their coordinates differ by at most 1 per direction.  Leaf
//   level L: fixed by the options, or the shallowest level whose mean
//   occupancy is at most the requested blobs per leaf, or by default the level
//   with the fewest pair evaluations per product (direct pairs plus M2L pairs,
//   counted level by level from level 2 while they fall); never deeper than
//   the deepest level with a cell side >= 2a (so every
//   interpolated pair has r > 2a and stays off the overlap branch of the
//   tensor).  Interaction list of a cell at level l >= 2: the non-empty cells
//   whose parent is adjacent to its parent and which are not adjacent to it.
// Per product (all on the GPU, sorted by Morton key):
//   P2M  qhat^c_m = sum_{j in c} S^c_m(y_j) lam_j at the leaves;
//   M2M  the parent's qhat from its children's proxies (exact: the parent's
//        Lagrange polynomials have degree n-1 and the children interpolate
//        them exactly);
//   M2L  v^c_k = sum_{c' in IL(c)} sum_m M(t^c_k, s^c'_m) qhat^c'_m, matrix-free
//        with the FP32 pair function (one workgroup per cell, lane groups of
//        one lane per target proxy taking listed cells in turn, the source
//        proxies of each listed cell staged in LDS; a listed cell with fewer
//        blobs than proxies enters with its blobs, n^3 |c'| pairs instead of
//        n^6);
//   L2L  the children's v gain the parent's interpolant at their proxies;
//   near + L2P  direct sums over the adjacent leaves (hi/lo split positions,
//        float runs promoted to double, as in the dense FP32 kernel) plus
//        sum_k S^leaf_k(x_i) v^leaf_k, written in the original blob order.
// With L <= 1 there is no interaction list: one cell, the direct sum.
// Single-blob bodies (Sec. 2.4): the generalised tensor, with the forces and
// the torques / a in two channels through P2M, M2M and L2L; M2L and the near
// field apply the 6 x 6 tensor between them.
// Two arithmetic variants share the tree and the float-rounded kernel values
// and weights: A = float (lambda, qhat and the runs of sums in float) and
// A = double (lambda, qhat and every sum in double).  The second is linear in
// lambda to double rounding, so Krylov iterations on it converge to any
// tolerance; the float variant serves the inner iterations of FP64 iterative
// refinement.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <memory>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <system_error>
#include <thread>
#include <type_traits>

#include "rot_device.h"

namespace arb {

namespace {

constexpr int kTabNode = 0, kTabDen = kFmmMaxOrder, kTabT1 = 2 * kFmmMaxOrder;
constexpr int kTabSize = 2 * kFmmMaxOrder + 2 * kFmmMaxOrder * kFmmMaxOrder;
constexpr int kNearBlock = 64;
constexpr int kFmmRun = 32;

template <class A>
using Vec4 = std::conditional_t<std::is_same_v<A, float>, float4, double4>;

template <class A>
__device__ __forceinline__ Vec4<A> vec4(A x, A y, A z) {
    Vec4<A> r;
    r.x = x;
    r.y = y;
    r.z = z;
    r.w = A(0);
    return r;
}

// free-space RPY coefficients c1, c2 (units of a) of M = c1 I + c2 r r^T
__device__ __forceinline__ void free_coef(float r2, float rinv, float &c1, float &c2) {
    constexpr CoefF c = kUnitCoefF;
    const float rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
    c1 = fmaf(c.k1, rinv3, rinv);
    c2 = fmaf(-c.k2, rinv3 * rinv2, rinv3);
    ARB_IF_ANY_OVERLAP(r2 <= c.four_a2)
    if (r2 <= c.four_a2) {
        const float rv = r2 > 0.f ? rinv : 0.f;
        c1 = fmaf(-c.n2, r2 * rv, c.n1);
        c2 = rv * c.n3;
    }
    ARB_END_IF_ANY
}

// acc += M(d) l for one pair: tensor coefficients in float, applied in A
template <bool WALL, class A>
__device__ __forceinline__ void pair_acc(float dx, float dy, float dz, float dxy2,
                                         const TargetZ<float> &zsc, float zi, float zj, float h2,
                                         float mh22, A lx, A ly, A lz, A &ax, A &ay, A &az) {
    constexpr CoefF cf = kUnitCoefF;
    const float r2 = fmaf(dz, dz, dxy2);
    const float rinv = rsq_f32(r2);
    if constexpr (WALL) {
        const float Rz = zi + zj;
        const float Ri = rsq_f32(fmaf(Rz, Rz, dxy2));
        const PairCoef<float> pc =
            wall_pair_coef<float>(r2, rinv, dxy2, zsc, zj, h2, mh22, Rz, Ri, cf);
        if constexpr (std::is_same_v<A, float>) {
            wall_pair_apply<float>(pc, pc.c, pc.d, dx, dy, dz, Rz, lx, ly, lz, ax, ay, az);
        } else {
            const PairCoef<double> pd{pc.cA, pc.cAe, pc.c2, pc.b, pc.c, pc.d, pc.e, pc.h2};
            wall_pair_apply<double>(pd, pd.c, pd.d, dx, dy, dz, Rz, lx, ly, lz, ax, ay, az);
        }
    } else {
        float c1, c2;
        free_coef(r2, rinv, c1, c2);
        const A rl = fma((A)dx, lx, fma((A)dy, ly, (A)dz * lz));
        const A t = (A)c2 * rl;
        ax = fma((A)c1, lx, fma(t, (A)dx, ax));
        ay = fma((A)c1, ly, fma(t, (A)dy, ay));
        az = fma((A)c1, lz, fma(t, (A)dz, az));
    }
}

struct Geo {
    double ox, oy, oz, S;  // root cube in units of a
    int n, P;
};

__device__ __forceinline__ void load_tab(const float *__restrict__ g, float *tab) {
    for (int i = threadIdx.x; i < kTabSize; i += blockDim.x) tab[i] = g[i];
    __syncthreads();
}

// the item of this workgroup when the launch has round_up(items, 8 kXcdChunk)
// workgroups: consecutive workgroups are dealt round-robin to the 8 XCDs, so
// this gives each XCD runs of kXcdChunk consecutive items (neighbouring cells in
// Morton order, which read the same leaves and multipole weights, share its
// L2), the runs dealt round-robin to keep the XCDs' loads even; -1 past the end
constexpr int kXcdChunk = 16;
__device__ __forceinline__ int xcd_item(int items) {
    const int x = blockIdx.x % 8, j = blockIdx.x / 8;
    const int it = (j / kXcdChunk) * 8 * kXcdChunk + x * kXcdChunk + j % kXcdChunk;
    return it < items ? it : -1;
}

// Lagrange polynomial l_k(u) at the Chebyshev points (product form)
__device__ __forceinline__ float lag(const float *tab, int n, int k, float u) {
    float p = tab[kTabDen + k];
    for (int j = 0; j < n; ++j)
        if (j != k) p *= u - tab[kTabNode + j];
    return p;
}

// a double split into float hi + lo
struct F2 {
    float h, l;
};
__device__ __forceinline__ F2 split(double x) {
    const float h = (float)x;
    return F2{h, (float)(x - (double)h)};
}

__device__ __forceinline__ double centre(double o, double side, int i) {
    return o + ((double)i + 0.5) * side;
}

// v of the cells of split interaction lists: the parts' sums, added in the
// order of the parts (m values of 3 P doubles per cell)
__global__ void fmm_split_sum_kernel(int64_t m, int splits, int P3,
                                     const double *__restrict__ vpart, double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t c = i / P3, r = i - c * P3;
    const double *p = vpart + c * splits * P3 + r;
    double t = 0.0;
    for (int j = 0; j < splits; ++j) t += p[(int64_t)j * P3];
    v[i] = t;
}

__global__ void fmm_sort_pos_kernel(int N, const int *__restrict__ perm,
                                    const float4 *__restrict__ hi, const float4 *__restrict__ lo,
                                    float4 *__restrict__ shi, float4 *__restrict__ slo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int i = perm[k];
    shi[k] = hi[i];
    slo[k] = lo[i];
}

template <class A>
__global__ void fmm_gather_lam_kernel(int N, const int *__restrict__ perm,
                                      const double *__restrict__ lam, Vec4<A> *__restrict__ slam) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int i = perm[k];
    slam[k] = vec4<A>((A)lam[3 * i], (A)lam[3 * i + 1], (A)lam[3 * i + 2]);
}

// qhat of the leaves, one workgroup per leaf, one lane per proxy: the leaf's
// blobs are staged in LDS in chunks with their 1D Lagrange values, computed
// once per blob and direction
constexpr int kP2MChunk = 64;

template <class A>
__global__ __launch_bounds__(kFmmMaxP) void fmm_p2m_kernel(
    Geo g, const float *__restrict__ tabg, const int4 *__restrict__ cc,
    const int2 *__restrict__ rng, int cell0, const float4 *__restrict__ shi,
    const float4 *__restrict__ slo, const Vec4<A> *__restrict__ slam, Vec4<A> *__restrict__ qhat) {
    __shared__ float tab[kTabSize];
    __shared__ float s_l[3][kP2MChunk][kFmmMaxOrder];
    __shared__ Vec4<A> s_lam[kP2MChunk];
    load_tab(tabg, tab);
    const int c = cell0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int n = g.n;
    const bool act = tid < g.P;
    const int k = act ? tid : 0;
    const int kx = k / (n * n), ky = (k / n) % n, kz = k % n;
    const int4 ci = cc[c];
    const int2 r = rng[c];
    const double side = ldexp(g.S, -ci.w);
    const F2 cd[3] = {split(centre(g.ox, side, ci.x)), split(centre(g.oy, side, ci.y)),
                      split(centre(g.oz, side, ci.z))};
    const float iw = (float)(2.0 / side);
    double qx = 0.0, qy = 0.0, qz = 0.0;
    for (int j0 = r.x; j0 < r.y; j0 += kP2MChunk) {
        const int cnt = min(kP2MChunk, r.y - j0);
        __syncthreads();
        for (int t = tid; t < 3 * cnt; t += blockDim.x) {
            const int jj = t / 3, d = t - 3 * jj;
            const float4 h = shi[j0 + jj], l = slo[j0 + jj];
            const float hx = d == 0 ? h.x : (d == 1 ? h.y : h.z);
            const float lx = d == 0 ? l.x : (d == 1 ? l.y : l.z);
            const float u = ((hx - cd[d].h) + (lx - cd[d].l)) * iw;
            for (int kk = 0; kk < n; ++kk) s_l[d][jj][kk] = lag(tab, n, kk, u);
            if (d == 0) s_lam[jj] = slam[j0 + jj];
        }
        __syncthreads();
        A fx = 0, fy = 0, fz = 0;
        for (int jj = 0; jj < cnt; ++jj) {
            const A w = (A)(s_l[0][jj][kx] * s_l[1][jj][ky] * s_l[2][jj][kz]);
            const Vec4<A> L = s_lam[jj];
            fx = fma(w, L.x, fx);
            fy = fma(w, L.y, fy);
            fz = fma(w, L.z, fz);
        }
        qx += fx;
        qy += fy;
        qz += fz;
    }
    if (act) qhat[(size_t)c * g.P + k] = vec4<A>((A)qx, (A)qy, (A)qz);
}

// qhat of the cells of one level from their children (NO points per direction)
template <class A, int NO>
__global__ __launch_bounds__(kFmmMaxP) void fmm_m2m_kernel(Geo g, const float *__restrict__ tabg,
                                                           const int4 *__restrict__ cc,
                                                           const int2 *__restrict__ kids,
                                                           int cell0, Vec4<A> *__restrict__ qhat) {
    __shared__ float tab[kTabSize];
    __shared__ Vec4<A> sq[kFmmMaxP];  // one child's weights, read by every lane
    load_tab(tabg, tab);
    const int c = cell0 + blockIdx.x;
    const int k = threadIdx.x;
    constexpr int n = NO, P = NO * NO * NO;
    const bool act = k < P;
    const int kx = k / (n * n), ky = (k / n) % n, kz = k % n;
    const int2 kr = kids[c];
    double qx = 0.0, qy = 0.0, qz = 0.0;
    for (int ch = kr.x; ch < kr.y; ++ch) {
        __syncthreads();
        if (act) sq[k] = qhat[(size_t)ch * P + k];
        __syncthreads();
        if (!act) continue;
        const int4 cci = cc[ch];
        // t1[sigma][k][m] = l_k(sigma/2 + xi_m/2): the parent's polynomial at the
        // child's proxies (sigma = -1 for the lower child, the even coordinate)
        const float *tx = tab + kTabT1 + (cci.x & 1) * kFmmMaxOrder * kFmmMaxOrder + kx * kFmmMaxOrder;
        const float *ty = tab + kTabT1 + (cci.y & 1) * kFmmMaxOrder * kFmmMaxOrder + ky * kFmmMaxOrder;
        const float *tz = tab + kTabT1 + (cci.z & 1) * kFmmMaxOrder * kFmmMaxOrder + kz * kFmmMaxOrder;
        const Vec4<A> *q = sq;
        A fx = 0, fy = 0, fz = 0;
        for (int mx = 0; mx < n; ++mx)
#pragma unroll
            for (int my = 0; my < n; ++my) {
                const float a = tx[mx] * ty[my];
#pragma unroll
                for (int mz = 0; mz < n; ++mz) {
                    const A w = (A)(a * tz[mz]);
                    const Vec4<A> Q = q[(mx * n + my) * n + mz];
                    fx = fma(w, Q.x, fx);
                    fy = fma(w, Q.y, fy);
                    fz = fma(w, Q.z, fz);
                }
            }
        qx += fx;
        qy += fy;
        qz += fz;
    }
    if (act) qhat[(size_t)c * P + k] = vec4<A>((A)qx, (A)qy, (A)qz);
}

// v of every cell of levels 2..L over its interaction list: `groups` lane
// groups of P (one lane per target proxy) take interaction-list entries in
// turn, so that groups * P fills the workgroup's waves; the groups' sums meet
// in LDS at the end
template <bool WALL, class A>
__global__ __launch_bounds__(kFmmMaxP) void fmm_m2l_kernel(
    Geo g, const float *__restrict__ tabg, const int4 *__restrict__ cc,
    const int *__restrict__ il_ptr, const int *__restrict__ il, int cell0, int items, int groups,
    int splits,
    const int2 *__restrict__ rng, const float4 *__restrict__ shi, const float4 *__restrict__ slo,
    const Vec4<A> *__restrict__ slam, const Vec4<A> *__restrict__ qhat, double *__restrict__ v,
    double *__restrict__ vpart) {
    const int item = xcd_item(items);
    if (item < 0) return;
    // LDS sized by the host: the sources of `groups` listed cells (offsets from
    // the cell's centre and charges), the groups' sums, the table
    extern __shared__ __align__(16) unsigned char lds[];
    const int n = g.n, P = g.P;
    const int GP = groups * P;  // <= kFmmMaxP
    Vec4<A> *s_q = reinterpret_cast<Vec4<A> *>(lds);
    float4 *s_off = reinterpret_cast<float4 *>(s_q + GP);
    double *s_acc = reinterpret_cast<double *>(s_off + GP);
    float *tab = reinterpret_cast<float *>(s_acc + 3 * (GP - P));
    load_tab(tabg, tab);
    // a cell's interaction list may be split over `splits` consecutive items,
    // each of which stores its part's sum at its own place in vpart
    const int c = cell0 + item / splits, part = item % splits;
    const int tid = threadIdx.x;
    const int4 ct = cc[c];
    const double side = ldexp(g.S, -ct.w), w = 0.5 * side;
    const bool act = tid < GP;
    const int gi = act ? tid / P : 0;
    const int k = act ? tid - gi * P : 0;
    const int kx = k / (n * n), ky = (k / n) % n, kz = k % n;
    const float okx = (float)(w * tab[kTabNode + kx]), oky = (float)(w * tab[kTabNode + ky]),
                okz = (float)(w * tab[kTabNode + kz]);
    const double czt = centre(g.oz, side, ct.z);
    const float zi = (float)(czt + w * tab[kTabNode + kz]);  // target proxy height
    const TargetZ<float> zsc = target_z(zi);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    const int b0 = il_ptr[c], len = il_ptr[c + 1] - b0;
    const int e1 = b0 + (int)((int64_t)len * (part + 1) / splits);
    for (int e0 = b0 + (int)((int64_t)len * part / splits); e0 < e1; e0 += groups) {
        __syncthreads();
        // a listed cell with fewer blobs than proxies enters with its blobs,
        // the others with their proxies (offsets w xi) and multipole weights
        for (int t = tid; t < GP; t += blockDim.x) {
            const int gg = t / P, m = t - gg * P;
            if (e0 + gg >= e1) continue;
            const int sc = il[e0 + gg];
            const int2 r = rng[sc];
            if (r.y - r.x < P) {
                if (m < r.y - r.x) {
                    const int4 cs = cc[sc];
                    const F2 cx = split(centre(g.ox, side, cs.x)),
                             cy = split(centre(g.oy, side, cs.y)),
                             cz = split(centre(g.oz, side, cs.z));
                    const float4 h = shi[r.x + m], l = slo[r.x + m];
                    s_off[t] = make_float4((h.x - cx.h) + (l.x - cx.l), (h.y - cy.h) + (l.y - cy.l),
                                           (h.z - cz.h) + (l.z - cz.l), 0.f);
                    s_q[t] = slam[r.x + m];
                }
            } else {
                const int mx = m / (n * n), my = (m / n) % n, mz = m % n;
                s_off[t] = make_float4((float)(w * tab[kTabNode + mx]),
                                       (float)(w * tab[kTabNode + my]),
                                       (float)(w * tab[kTabNode + mz]), 0.f);
                s_q[t] = qhat[(size_t)sc * P + m];
            }
        }
        __syncthreads();
        const int e = e0 + gi;
        if (!act || e >= e1) continue;
        const int sc = il[e];
        const int4 cs = cc[sc];
        const int cnt = min(P, rng[sc].y - rng[sc].x);
        // target proxy minus source cell centre, from the integer offset
        const float ax = (float)((double)(ct.x - cs.x) * side) + okx;
        const float ay = (float)((double)(ct.y - cs.y) * side) + oky;
        const float az = (float)((double)(ct.z - cs.z) * side) + okz;
        const float zc = (float)centre(g.oz, side, cs.z);
        const float4 *so = s_off + gi * P;
        const Vec4<A> *sq = s_q + gi * P;
        for (int m0 = 0; m0 < cnt; m0 += kFmmRun) {
            const int m1 = min(m0 + kFmmRun, cnt);
            A fx = 0, fy = 0, fz = 0;
            for (int m = m0; m < m1; ++m) {
                const float4 o = so[m];
                const Vec4<A> q = sq[m];
                const float dx = ax - o.x, dy = ay - o.y, dz = az - o.z;
                const float dxy2 = fmaf(dx, dx, dy * dy);
                const float zj = zc + o.z;
                const float h2 = 2.f * zj;
                pair_acc<WALL, A>(dx, dy, dz, dxy2, zsc, zi, zj, h2, -(h2 * h2), q.x, q.y, q.z, fx,
                                  fy, fz);
            }
            ux += fx;
            uy += fy;
            uz += fz;
        }
    }
    // the groups' sums, added in group order
    __syncthreads();
    if (act && gi > 0) {
        double *a = s_acc + 3 * (tid - P);
        a[0] = ux;
        a[1] = uy;
        a[2] = uz;
    }
    __syncthreads();
    if (act && gi == 0) {
        for (int gg = 1; gg < groups; ++gg) {
            const double *a = s_acc + 3 * ((gg - 1) * P + k);
            ux += a[0];
            uy += a[1];
            uz += a[2];
        }
        double *o = splits == 1 ? v + ((size_t)c * P + k) * 3 : vpart + ((size_t)item * P + k) * 3;
        o[0] = ux;
        o[1] = uy;
        o[2] = uz;
    }
}

// the children at one level gain the parent's interpolant at their proxies (NO
// points per direction)
template <int NO>
__global__ __launch_bounds__(kFmmMaxP) void fmm_l2l_kernel(Geo g, const float *__restrict__ tabg,
                                                           const int4 *__restrict__ cc,
                                                           const int *__restrict__ parent,
                                                           int cell0, double *__restrict__ v) {
    __shared__ float tab[kTabSize];
    __shared__ double sv[3 * kFmmMaxP];  // the parent's values, read by every lane
    load_tab(tabg, tab);
    const int c = cell0 + blockIdx.x;
    const int m = threadIdx.x;
    constexpr int n = NO, P = NO * NO * NO;
    {
        const double *vp = v + (size_t)parent[c] * P * 3;
        for (int i = m; i < 3 * P; i += blockDim.x) sv[i] = vp[i];
    }
    __syncthreads();
    if (m >= P) return;
    const int mx = m / (n * n), my = (m / n) % n, mz = m % n;
    const int4 cci = cc[c];
    const float *tx = tab + kTabT1 + (cci.x & 1) * kFmmMaxOrder * kFmmMaxOrder + mx;
    const float *ty = tab + kTabT1 + (cci.y & 1) * kFmmMaxOrder * kFmmMaxOrder + my;
    const float *tz = tab + kTabT1 + (cci.z & 1) * kFmmMaxOrder * kFmmMaxOrder + mz;
    const double *vp = sv;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int kx = 0; kx < n; ++kx)
#pragma unroll
        for (int ky = 0; ky < n; ++ky) {
            const double a = (double)(tx[kx * kFmmMaxOrder] * ty[ky * kFmmMaxOrder]);
#pragma unroll
            for (int kz = 0; kz < n; ++kz) {
                const double wk = a * (double)tz[kz * kFmmMaxOrder];
                const double *pv = vp + 3 * ((kx * n + ky) * n + kz);
                sx = fma(wk, pv[0], sx);
                sy = fma(wk, pv[1], sy);
                sz = fma(wk, pv[2], sz);
            }
        }
    double *o = v + ((size_t)c * P + m) * 3;
    o[0] += sx;
    o[1] += sy;
    o[2] += sz;
}

// direct sums over the adjacent leaves plus the leaf's interpolant; one
// workgroup per (leaf, run of 64 targets); output in the original blob order
template <bool WALL, class A>
__global__ __launch_bounds__(kNearBlock) void fmm_near_kernel(
    Geo g, const float *__restrict__ tabg, int N, int far, const int4 *__restrict__ cc,
    const int2 *__restrict__ rng, const int *__restrict__ near_ptr, const int *__restrict__ near,
    int leaf0, const int2 *__restrict__ work, int items, const int *__restrict__ perm,
    const float4 *__restrict__ shi, const float4 *__restrict__ slo,
    const Vec4<A> *__restrict__ slam, const double *__restrict__ v, double *__restrict__ partial) {
    const int item = xcd_item(items);
    if (item < 0) return;
    __shared__ float tab[kTabSize];
    __shared__ float4 s_hi[kNearBlock], s_lo[kNearBlock];
    __shared__ Vec4<A> s_lam[kNearBlock];
    load_tab(tabg, tab);
    const int tid = threadIdx.x;
    const int2 wk = work[item];
    const int c = wk.x;
    const int2 tr = rng[c];
    const int i = wk.y + tid;
    const bool act = i < tr.y;
    const int ic = act ? i : tr.y - 1;
    const float4 th = shi[ic], tl = slo[ic];
    const float zi = th.z + tl.z;
    const TargetZ<float> zsc = target_z(zi);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    const int lf = c - leaf0;
    const int e1 = near_ptr[lf + 1];
    for (int e = near_ptr[lf]; e < e1; ++e) {
        const int2 sr = rng[near[e]];
        for (int j0 = sr.x; j0 < sr.y; j0 += kNearBlock) {
            const int j = j0 + tid;
            __syncthreads();
            if (j < sr.y) {
                s_hi[tid] = shi[j];
                s_lo[tid] = slo[j];
                s_lam[tid] = slam[j];
            }
            __syncthreads();
            const int cnt = min(kNearBlock, sr.y - j0);
            for (int k0 = 0; k0 < cnt; k0 += kFmmRun) {
                const int k1 = min(k0 + kFmmRun, cnt);
                A ax = 0, ay = 0, az = 0;
                for (int k = k0; k < k1; ++k) {
                    const float4 sh = s_hi[k], sl = s_lo[k];
                    const Vec4<A> L = s_lam[k];
                    const float dx = (th.x - sh.x) + (tl.x - sl.x);
                    const float dy = (th.y - sh.y) + (tl.y - sl.y);
                    const float dz = (th.z - sh.z) + (tl.z - sl.z);
                    const float dxy2 = fmaf(dx, dx, dy * dy);
                    pair_acc<WALL, A>(dx, dy, dz, dxy2, zsc, zi, sh.z, sh.w, sl.w, L.x, L.y, L.z,
                                      ax, ay, az);
                }
                ux += ax;
                uy += ay;
                uz += az;
            }
        }
    }
    if (far) {
        const int n = g.n;
        const int4 ci = cc[c];
        const double side = ldexp(g.S, -ci.w);
        const F2 cx = split(centre(g.ox, side, ci.x)), cy = split(centre(g.oy, side, ci.y)),
                 cz = split(centre(g.oz, side, ci.z));
        const float iw = (float)(2.0 / side);
        const float px = ((th.x - cx.h) + (tl.x - cx.l)) * iw;
        const float py = ((th.y - cy.h) + (tl.y - cy.l)) * iw;
        const float pz = ((th.z - cz.h) + (tl.z - cz.l)) * iw;
        const double *vc = v + (size_t)c * g.P * 3;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int kx = 0; kx < n; ++kx) {
            const float a = lag(tab, n, kx, px);
            for (int ky = 0; ky < n; ++ky) {
                const float b = a * lag(tab, n, ky, py);
                for (int kz = 0; kz < n; ++kz) {
                    const double wk = (double)(b * lag(tab, n, kz, pz));
                    const double *pv = vc + 3 * ((kx * n + ky) * n + kz);
                    sx = fma(wk, pv[0], sx);
                    sy = fma(wk, pv[1], sy);
                    sz = fma(wk, pv[2], sz);
                }
            }
        }
        ux += sx;
        uy += sy;
        uz += sz;
    }
    if (act) {
        const size_t o = (size_t)perm[i];
        partial[o] = ux;
        partial[(size_t)N + o] = uy;
        partial[2 * (size_t)N + o] = uz;
    }
}

// ---------------------------------------------------------------- single-blob bodies
// Generalised forces (f, tau) in two channels, f and tau / a (units of a), each
// carried by the channel-wise P2M, M2M and L2L kernels above; M2L and the near
// field apply the 6 x 6 generalised tensor (Sec. 2.4) between the channels.

template <class A>
__global__ void fmm_gather6_kernel(int M, const int *__restrict__ perm,
                                   const double *__restrict__ x6, double inv_a,
                                   Vec4<A> *__restrict__ sf, Vec4<A> *__restrict__ st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const double *x = x6 + 6 * (size_t)perm[k];
    sf[k] = vec4<A>((A)x[0], (A)x[1], (A)x[2]);
    st[k] = vec4<A>((A)(x[3] * inv_a), (A)(x[4] * inv_a), (A)(x[5] * inv_a));
}

// acc += N(d) (f, t): tensor coefficients in float (a = 1), applied in A
template <class A>
__device__ __forceinline__ void rot_acc(float dx, float dy, float dz, float r2, const Vec4<A> &f,
                                        const Vec4<A> &t, A *acc) {
    const float rinv = rsq_f32(r2);
    const RotTerms<float> kf = rot_terms<float>(r2, rinv, kUnitRotCoef);
    if constexpr (std::is_same_v<A, float>) {
        rot_one_way<float>(kf, dx, dy, dz, f.x, f.y, f.z, t.x, t.y, t.z, acc);
    } else {
        const RotTerms<double> kd{kf.c1, kf.c2, kf.cr, kf.d1, kf.d2};
        rot_one_way<double>(kd, dx, dy, dz, f.x, f.y, f.z, t.x, t.y, t.z, acc);
    }
}

// M2L of the generalised tensor (unbounded), lane groups as in fmm_m2l_kernel
template <class A>
__global__ __launch_bounds__(kFmmMaxP) void fmm_m2l6_kernel(
    Geo g, const float *__restrict__ tabg, const int4 *__restrict__ cc,
    const int *__restrict__ il_ptr, const int *__restrict__ il, int cell0, int items, int groups,
    int splits,
    const int2 *__restrict__ rng, const float4 *__restrict__ shi, const float4 *__restrict__ slo,
    const Vec4<A> *__restrict__ sf, const Vec4<A> *__restrict__ st,
    const Vec4<A> *__restrict__ qf, const Vec4<A> *__restrict__ qt, double *__restrict__ vu,
    double *__restrict__ vw, double *__restrict__ vpart) {
    const int item = xcd_item(items);
    if (item < 0) return;
    extern __shared__ __align__(16) unsigned char lds[];
    const int n = g.n, P = g.P;
    const int GP = groups * P;  // <= kFmmMaxP
    Vec4<A> *s_qf = reinterpret_cast<Vec4<A> *>(lds);
    Vec4<A> *s_qt = s_qf + GP;
    float4 *s_off = reinterpret_cast<float4 *>(s_qt + GP);
    double *s_acc = reinterpret_cast<double *>(s_off + GP);
    float *tab = reinterpret_cast<float *>(s_acc + 6 * (GP - P));
    load_tab(tabg, tab);
    // a cell's interaction list may be split over `splits` consecutive items,
    // each of which stores its part's sum at its own place in vpart
    const int c = cell0 + item / splits, part = item % splits;
    const int tid = threadIdx.x;
    const int4 ct = cc[c];
    const double side = ldexp(g.S, -ct.w), w = 0.5 * side;
    const bool act = tid < GP;
    const int gi = act ? tid / P : 0;
    const int k = act ? tid - gi * P : 0;
    const int kx = k / (n * n), ky = (k / n) % n, kz = k % n;
    const float okx = (float)(w * tab[kTabNode + kx]), oky = (float)(w * tab[kTabNode + ky]),
                okz = (float)(w * tab[kTabNode + kz]);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int b0 = il_ptr[c], len = il_ptr[c + 1] - b0;
    const int e1 = b0 + (int)((int64_t)len * (part + 1) / splits);
    for (int e0 = b0 + (int)((int64_t)len * part / splits); e0 < e1; e0 += groups) {
        __syncthreads();
        // sparse listed cells enter with their bodies, the others with proxies
        for (int t = tid; t < GP; t += blockDim.x) {
            const int gg = t / P, m = t - gg * P;
            if (e0 + gg >= e1) continue;
            const int sc = il[e0 + gg];
            const int2 r = rng[sc];
            if (r.y - r.x < P) {
                if (m < r.y - r.x) {
                    const int4 cs = cc[sc];
                    const F2 cx = split(centre(g.ox, side, cs.x)),
                             cy = split(centre(g.oy, side, cs.y)),
                             cz = split(centre(g.oz, side, cs.z));
                    const float4 h = shi[r.x + m], l = slo[r.x + m];
                    s_off[t] = make_float4((h.x - cx.h) + (l.x - cx.l), (h.y - cy.h) + (l.y - cy.l),
                                           (h.z - cz.h) + (l.z - cz.l), 0.f);
                    s_qf[t] = sf[r.x + m];
                    s_qt[t] = st[r.x + m];
                }
            } else {
                const int mx = m / (n * n), my = (m / n) % n, mz = m % n;
                s_off[t] = make_float4((float)(w * tab[kTabNode + mx]),
                                       (float)(w * tab[kTabNode + my]),
                                       (float)(w * tab[kTabNode + mz]), 0.f);
                const size_t q = (size_t)sc * P + m;
                s_qf[t] = qf[q];
                s_qt[t] = qt[q];
            }
        }
        __syncthreads();
        const int e = e0 + gi;
        if (!act || e >= e1) continue;
        const int sc = il[e];
        const int4 cs = cc[sc];
        const int cnt = min(P, rng[sc].y - rng[sc].x);
        const float ax = (float)((double)(ct.x - cs.x) * side) + okx;
        const float ay = (float)((double)(ct.y - cs.y) * side) + oky;
        const float az = (float)((double)(ct.z - cs.z) * side) + okz;
        const Vec4<A> *qfg = s_qf + gi * P, *qtg = s_qt + gi * P;
        const float4 *so = s_off + gi * P;
        for (int m0 = 0; m0 < cnt; m0 += kFmmRun) {
            const int m1 = min(m0 + kFmmRun, cnt);
            A f6[6] = {0, 0, 0, 0, 0, 0};
            for (int m = m0; m < m1; ++m) {
                const float4 o = so[m];
                const float dx = ax - o.x, dy = ay - o.y, dz = az - o.z;
                rot_acc<A>(dx, dy, dz, fmaf(dz, dz, fmaf(dx, dx, dy * dy)), qfg[m], qtg[m], f6);
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) acc[j] += f6[j];
        }
    }
    __syncthreads();
    if (act && gi > 0) {
#pragma unroll
        for (int j = 0; j < 6; ++j) s_acc[6 * (tid - P) + j] = acc[j];
    }
    __syncthreads();
    if (act && gi == 0) {
        for (int gg = 1; gg < groups; ++gg)
#pragma unroll
            for (int j = 0; j < 6; ++j) acc[j] += s_acc[6 * ((gg - 1) * P + k) + j];
        double *ou, *ow;
        if (splits == 1) {
            ou = vu + ((size_t)c * P + k) * 3;
            ow = vw + ((size_t)c * P + k) * 3;
        } else {
            ou = vpart + ((size_t)item * P + k) * 3;
            ow = ou + (size_t)items * P * 3;
        }
        ou[0] = acc[0];
        ou[1] = acc[1];
        ou[2] = acc[2];
        ow[0] = acc[3];
        ow[1] = acc[4];
        ow[2] = acc[5];
    }
}

// direct sums of the generalised tensor over adjacent leaves plus both
// channels' interpolants; partial[j][body] (6 x M, original order)
template <class A>
__global__ __launch_bounds__(kNearBlock) void fmm_near6_kernel(
    Geo g, const float *__restrict__ tabg, int M, int far, const int4 *__restrict__ cc,
    const int2 *__restrict__ rng, const int *__restrict__ near_ptr, const int *__restrict__ near,
    int leaf0, const int2 *__restrict__ work, int items, const int *__restrict__ perm,
    const float4 *__restrict__ shi, const float4 *__restrict__ slo, const Vec4<A> *__restrict__ sf,
    const Vec4<A> *__restrict__ st, const double *__restrict__ vu, const double *__restrict__ vw,
    double *__restrict__ partial) {
    const int item = xcd_item(items);
    if (item < 0) return;
    __shared__ float tab[kTabSize];
    __shared__ float4 s_hi[kNearBlock], s_lo[kNearBlock];
    __shared__ Vec4<A> s_f[kNearBlock], s_t[kNearBlock];
    load_tab(tabg, tab);
    const int tid = threadIdx.x;
    const int2 wk = work[item];
    const int c = wk.x;
    const int2 tr = rng[c];
    const int i = wk.y + tid;
    const bool act = i < tr.y;
    const int ic = act ? i : tr.y - 1;
    const float4 th = shi[ic], tl = slo[ic];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int lf = c - leaf0;
    const int e1 = near_ptr[lf + 1];
    for (int e = near_ptr[lf]; e < e1; ++e) {
        const int2 sr = rng[near[e]];
        for (int j0 = sr.x; j0 < sr.y; j0 += kNearBlock) {
            const int j = j0 + tid;
            __syncthreads();
            if (j < sr.y) {
                s_hi[tid] = shi[j];
                s_lo[tid] = slo[j];
                s_f[tid] = sf[j];
                s_t[tid] = st[j];
            }
            __syncthreads();
            const int cnt = min(kNearBlock, sr.y - j0);
            for (int k0 = 0; k0 < cnt; k0 += kFmmRun) {
                const int k1 = min(k0 + kFmmRun, cnt);
                A f6[6] = {0, 0, 0, 0, 0, 0};
                for (int k = k0; k < k1; ++k) {
                    const float4 sh = s_hi[k], sl = s_lo[k];
                    const float dx = (th.x - sh.x) + (tl.x - sl.x);
                    const float dy = (th.y - sh.y) + (tl.y - sl.y);
                    const float dz = (th.z - sh.z) + (tl.z - sl.z);
                    rot_acc<A>(dx, dy, dz, fmaf(dz, dz, fmaf(dx, dx, dy * dy)), s_f[k], s_t[k],
                               f6);
                }
#pragma unroll
                for (int jj = 0; jj < 6; ++jj) acc[jj] += f6[jj];
            }
        }
    }
    if (far) {
        const int n = g.n;
        const int4 ci = cc[c];
        const double side = ldexp(g.S, -ci.w);
        const F2 cx = split(centre(g.ox, side, ci.x)), cy = split(centre(g.oy, side, ci.y)),
                 cz = split(centre(g.oz, side, ci.z));
        const float iw = (float)(2.0 / side);
        const float px = ((th.x - cx.h) + (tl.x - cx.l)) * iw;
        const float py = ((th.y - cy.h) + (tl.y - cy.l)) * iw;
        const float pz = ((th.z - cz.h) + (tl.z - cz.l)) * iw;
        const double *pu = vu + (size_t)c * g.P * 3, *pw = vw + (size_t)c * g.P * 3;
        for (int kx = 0; kx < n; ++kx) {
            const float a = lag(tab, n, kx, px);
            for (int ky = 0; ky < n; ++ky) {
                const float b = a * lag(tab, n, ky, py);
                for (int kz = 0; kz < n; ++kz) {
                    const double wk2 = (double)(b * lag(tab, n, kz, pz));
                    const int q = 3 * ((kx * n + ky) * n + kz);
                    acc[0] = fma(wk2, pu[q], acc[0]);
                    acc[1] = fma(wk2, pu[q + 1], acc[1]);
                    acc[2] = fma(wk2, pu[q + 2], acc[2]);
                    acc[3] = fma(wk2, pw[q], acc[3]);
                    acc[4] = fma(wk2, pw[q + 1], acc[4]);
                    acc[5] = fma(wk2, pw[q + 2], acc[5]);
                }
            }
        }
    }
    if (act) {
        const size_t o = (size_t)perm[i];
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) partial[(size_t)jj * M + o] = acc[jj];
    }
}

// ---------------------------------------------------------------- host tree
inline uint64_t spread3(uint64_t x) {  // 21 bits -> every third bit
    x &= 0x1fffff;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
inline uint64_t morton(int x, int y, int z) {
    return (spread3((uint64_t)x) << 2) | (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
}
inline int compact3(uint64_t x) {  // every third bit -> 21 bits (inverse of spread3)
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x1f00000000ffffull;
    x = (x | (x >> 32)) & 0x1fffffull;
    return (int)x;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// host threads for the O(N) steps of the tree build: at most 16 (one GPU's
// share of the host), one per 65,536 blobs; the environment variable
// ARB_HOST_THREADS (1..16) caps them (the plan does not depend on the count)
int host_threads(int N) {
    int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    if (const char *e = std::getenv("ARB_HOST_THREADS")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 16) hw = std::min(hw, v);
    }
    return std::max(1, std::min({16, hw, N / 65536}));
}

// FNV-1a over the bytes of a vector
template <class V>
void fnv1a(uint64_t &h, const std::vector<V> &v) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(v.data());
    const size_t n = v.size() * sizeof(V);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
}

// Host worker threads kept for the life of the process (started on first use,
// at most 15), so that the tree build's many short parallel steps do not each
// start and join threads.  One job at a time: a caller that finds the pool busy
// (another context building its tree on another thread) gets false and runs
// the step on threads of its own.  The pool is never destroyed; its idle
// workers wait on a condition variable until the process ends.
class HostPool {
  public:
    // slice(t) for t in [0, T): t = 0 on the caller's thread, the others on
    // workers; slice must not throw.  False (nothing run) when the pool is busy
    // or cannot start enough workers.
    bool run(int T, const std::function<void(int)> &slice) {
        std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
        if (!busy.owns_lock()) return false;
        {
            std::lock_guard<std::mutex> lk(mu_);
            try {
                while ((int)workers_.size() < T - 1) {
                    const int id = (int)workers_.size() + 1;
                    workers_.emplace_back([this, id] { worker(id); });
                }
            } catch (const std::system_error &) {
                return false;
            }
            job_ = &slice;
            job_T_ = T;
            pending_ = T - 1;
            ++gen_;
        }
        cv_.notify_all();
        slice(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_.wait(lk, [this] { return pending_ == 0; });
        job_ = nullptr;
        return true;
    }

  private:
    void worker(int id) {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (id >= job_T_) continue;
            const std::function<void(int)> *f = job_;
            lk.unlock();
            (*f)(id);
            lk.lock();
            if (--pending_ == 0) done_.notify_one();
        }
    }
    std::mutex busy_, mu_;
    std::condition_variable cv_, done_;
    std::vector<std::thread> workers_;
    const std::function<void(int)> *job_ = nullptr;
    int job_T_ = 0, pending_ = 0;
    uint64_t gen_ = 0;
};

HostPool &host_pool() {
    static HostPool *pool = new HostPool;  // never freed (see above)
    return *pool;
}

// f(t, i0, i1) on T contiguous slices of [0, N), slice t on thread t (of the
// host pool, or of threads started for this step when the pool is busy).  An
// exception in a slice is caught on its thread and rethrown on the caller's
// after every slice has ended; a slice whose thread cannot be started runs on
// the caller's thread (the result does not depend on where a slice runs).
template <class F>
void parallel_slices(int T, int N, F &&f) {
    if (T <= 1) {
        f(0, 0, N);
        return;
    }
    std::vector<std::exception_ptr> err((size_t)T);
    const std::function<void(int)> slice = [&f, &err, T, N](int t) {
        const int i0 = (int)((int64_t)N * t / T), i1 = (int)((int64_t)N * (t + 1) / T);
        try {
            f(t, i0, i1);
        } catch (...) {
            err[t] = std::current_exception();
        }
    };
    if (!host_pool().run(T, slice)) {
        std::vector<std::thread> th;
        th.reserve(T);
        for (int t = 0; t < T; ++t) {
            try {
                th.emplace_back(slice, t);
            } catch (const std::system_error &) {
                slice(t);
            }
        }
        for (auto &x : th) x.join();
    }
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// per-cell lists on host threads: f(c, out) appends the entries of item c to
// out for c in [0, n); ptr gets the prefix sums of their counts and out the
// entries joined in item order, as a loop over the items would give them
template <class V, class F>
void lists_by_item(int threads, int n, std::vector<int> &ptr, std::vector<V> &out, F &&f) {
    const int T = std::max(1, std::min(threads, n / 256));
    std::vector<std::vector<V>> part((size_t)T);
    ptr.assign((size_t)n + 1, 0);
    parallel_slices(T, n, [&](int t, int c0, int c1) {
        std::vector<V> &v = part[t];
        for (int c = c0; c < c1; ++c) {
            const size_t before = v.size();
            f(c, v);
            ptr[c + 1] = (int)(v.size() - before);
        }
    });
    for (int c = 0; c < n; ++c) ptr[c + 1] += ptr[c];
    out.clear();
    out.reserve((size_t)ptr[n]);
    for (const std::vector<V> &v : part) out.insert(out.end(), v.begin(), v.end());
}

// open-addressing map from the Morton keys of one level's cells (< 2^48) to
// their indices
struct CellHash {
    std::vector<uint64_t> keys;
    std::vector<int> vals;
    uint64_t mask = 0;
    static uint64_t mix(uint64_t x) {
        x ^= x >> 30;
        x *= 0xbf58476d1ce4e5b9ull;
        x ^= x >> 27;
        x *= 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    }
    // the keys k[0..n) (distinct) with values base + i; up to `threads` host
    // threads claim slots with compare-and-swap, so the table's layout may depend
    // on their timing, but every lookup finds the same value
    void build(const uint64_t *k, int n, int base, int threads);
    // index of the cell with coordinates (x, y, z) at a level of side 2^l, or -1
    int get(int l, int x, int y, int z) const {
        const int lim = 1 << l;
        if (x < 0 || y < 0 || z < 0 || x >= lim || y >= lim || z >= lim) return -1;
        const uint64_t k = morton(x, y, z);
        for (uint64_t h = mix(k) & mask; keys[h] != ~0ull; h = (h + 1) & mask)
            if (keys[h] == k) return vals[h];
        return -1;
    }
};

void CellHash::build(const uint64_t *k, int n, int base, int threads) {
    size_t cap = 16;
    while (cap < 2 * (size_t)n) cap *= 2;
    mask = cap - 1;
    keys.assign(cap, ~0ull);
    vals.assign(cap, -1);
    const int T = std::max(1, std::min(threads, n / 16384));
    parallel_slices(T, n, [&](int, int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            uint64_t h = mix(k[i]) & mask;
            for (;;) {
                uint64_t empty = ~0ull;
                if (__atomic_compare_exchange_n(&keys[h], &empty, k[i], false, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED)) {
                    vals[h] = base + i;
                    break;
                }
                h = (h + 1) & mask;
            }
        }
    });
}

// work items per cell in M2L: one, or up to 8 when there are too few cells to
// fill the chip (about 2,048 items wanted)
int m2l_splits(int cells) {
    return std::max(1, std::min(8, (2048 + cells - 1) / std::max(cells, 1)));
}

// calls f with the order n (2..kFmmMaxOrder, checked when the options are
// read) as a compile-time constant, for the kernels whose loops unroll over it
template <class F> void with_order(int n, F &&f) {
    static_assert(kFmmMaxOrder == 8, "cases 2..8");
    switch (n) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
    }
}

// M2L lane groups per workgroup: the count (up to 8 within 512 lanes) that
// leaves the fewest idle lanes in its waves
int m2l_groups(int P) {
    int groups = 1;
    double best = 0.0;
    for (int gq = 1; gq <= 8 && gq * P <= kFmmMaxP; ++gq) {
        const double util = (double)(gq * P) / round_up(gq * P, kWave);
        if (util > best + 1e-9) {
            best = util;
            groups = gq;
        }
    }
    return groups;
}

}  // namespace

// the octree of N positions (units of length, host memory), built on the host
struct FmmPlan {
    int n = 0, P = 0, L = 0, ncell = 0, nleaf = 0;
    double o[3] = {0.0, 0.0, 0.0}, S = 0.0;  // root cube, units of length
    int64_t n_near_pairs = 0, n_m2l_pairs = 0;
    std::vector<int> perm, lvl, parent, il_ptr, il, near_ptr, nearl;
    std::vector<int4> cc;
    std::vector<int2> rng, kids, work;
    std::vector<float> tab;
};

// Host scratch of the tree build: grow-only arrays whose contents are not
// initialised (every entry used is written first), kept between builds so that
// their pages are allocated and touched once
template <class T>
struct HostArr {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    T *get(size_t m) {
        if (m > n || !p) {
            p.reset(new T[std::max<size_t>(m, 1)]);
            n = std::max<size_t>(m, 1);
        }
        return p.get();
    }
};
struct PlanScratch {
    HostArr<int> crd, idx, idx2;
    HostArr<uint64_t> key, key2;
    HostArr<unsigned char> first;
};

}  // namespace arb

// what a context keeps of its tree builds: the scratch, the last plan (its
// vectors' capacity is reused) and pinned host memory for the positions
struct arb::FmmHostCache {
    PlanScratch scratch;
    FmmPlan plan;
    double *hpos = nullptr;
    size_t hpos_n = 0;
    FmmHostCache() = default;
    FmmHostCache(const FmmHostCache &) = delete;
    FmmHostCache &operator=(const FmmHostCache &) = delete;
    ~FmmHostCache() {
        if (hpos) (void)hipHostFree(hpos);
    }
    // pinned room for n doubles (null when it cannot be allocated)
    double *positions(size_t n) {
        if (n <= hpos_n && hpos) return hpos;
        if (hpos) (void)hipHostFree(hpos);
        hpos = nullptr;
        hpos_n = 0;
        if (hipHostMalloc((void **)&hpos, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            hpos = nullptr;
            return nullptr;
        }
        hpos_n = n;
        return hpos;
    }
};

namespace arb {

int fmm_plan(FmmPlan &pl, PlanScratch &sc, int N, const double *h, double a, int n, int levels,
             int leaf, std::string *msg) {
    const int P = n * n * n;
    const int T = host_threads(N);
    // finite positions and the root cube (host threads over slices; min and max
    // are exact, so the result does not depend on the slicing)
    std::vector<double> bound(6 * (size_t)T);
    std::vector<char> bad((size_t)T, 0);
    parallel_slices(T, N, [&](int t, int i0, int i1) {
        // running bounds in registers, stored once (the threads' slots share
        // cache lines)
        double lo[3] = {h[0], h[1], h[2]}, up[3] = {h[0], h[1], h[2]};
        bool finite = true;
        for (int i = i0; i < i1; ++i)
            for (int d = 0; d < 3; ++d) {
                const double x = h[3 * (size_t)i + d];
                finite = finite && std::isfinite(x);
                lo[d] = std::min(lo[d], x);
                up[d] = std::max(up[d], x);
            }
        for (int d = 0; d < 3; ++d) {
            bound[6 * (size_t)t + d] = lo[d];
            bound[6 * (size_t)t + 3 + d] = up[d];
        }
        if (!finite) bad[t] = 1;
    });
    for (int t = 0; t < T; ++t)
        if (bad[t]) {
            *msg = "fast product: a position is not finite";
            return ARB_E_NAN;
        }
    double o[3] = {h[0], h[1], h[2]}, hi_d[3] = {h[0], h[1], h[2]}, ext = 0.0;
    for (int t = 0; t < T; ++t)
        for (int d = 0; d < 3; ++d) {
            o[d] = std::min(o[d], bound[6 * (size_t)t + d]);
            hi_d[d] = std::max(hi_d[d], bound[6 * (size_t)t + 3 + d]);
        }
    for (int d = 0; d < 3; ++d) ext = std::max(ext, hi_d[d] - o[d]);
    const double S = ext > 0.0 ? ext * (1.0 + 0x1p-20) : a;
    int Lhi = 0;  // deepest level with a cell side >= 2a
    while (Lhi < kFmmMaxLevel && S / std::ldexp(1.0, Lhi + 1) >= 2.0 * a) ++Lhi;
    // cell coordinates at level Lhi and Morton keys (host threads over slices;
    // the arrays are left uninitialised, so that their pages are first touched
    // by the threads that fill them)
    int *crd = sc.crd.get(3 * (size_t)N);
    uint64_t *key = sc.key.get(N), *key2 = sc.key2.get(N);
    int *idx = sc.idx.get(N), *idx2 = sc.idx2.get(N);
    const double scale = std::ldexp(1.0, Lhi);
    parallel_slices(T, N, [&](int, int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            int cq[3];
            for (int d = 0; d < 3; ++d) {
                const double u = (h[3 * (size_t)i + d] - o[d]) / S;
                cq[d] = (int)std::floor(u * scale);
                crd[3 * (size_t)i + d] = cq[d];
            }
            key[i] = morton(cq[0], cq[1], cq[2]);
            idx[i] = i;
        }
    });
    // stable LSD radix sort of the 3 Lhi-bit keys in the fewest passes of at
    // most 14 bits: blobs in Morton order, equal keys in ascending blob index.
    // Each thread counts and then scatters its own contiguous slice, at offsets
    // ordered by bucket and then by thread, which keeps the sort stable.
    {
        const int bits = 3 * Lhi, passes = (bits + 13) / 14;
        const int dbits = passes ? (bits + passes - 1) / passes : 0;
        const size_t B = (size_t)1 << dbits;
        const uint64_t mask = B - 1;
        std::vector<int> cnt((size_t)T * B);
        for (int ps = 0; ps < passes; ++ps) {
            const int shift = ps * dbits;
            parallel_slices(T, N, [&](int t, int i0, int i1) {
                int *c = cnt.data() + (size_t)t * B;
                std::fill(c, c + B, 0);
                for (int i = i0; i < i1; ++i) ++c[(key[i] >> shift) & mask];
            });
            int run = 0;
            for (size_t b = 0; b < B; ++b)
                for (int t = 0; t < T; ++t) {
                    const int m = cnt[(size_t)t * B + b];
                    cnt[(size_t)t * B + b] = run;
                    run += m;
                }
            parallel_slices(T, N, [&](int t, int i0, int i1) {
                int *c = cnt.data() + (size_t)t * B;
                for (int i = i0; i < i1; ++i) {
                    const int at = c[(key[i] >> shift) & mask]++;
                    key2[at] = key[i];
                    idx2[at] = idx[i];
                }
            });
            std::swap(key, key2);
            std::swap(idx, idx2);
        }
    }
    // the shallowest level at which sorted blob j starts a new cell (a cell
    // starts at every deeper level too): the highest differing key bit / 3
    unsigned char *first = sc.first.get(N);
    first[0] = 0;
    std::vector<int64_t> new_at_t((size_t)T * (Lhi + 2), 0), new_at(Lhi + 2, 0);
    parallel_slices(T, N, [&](int t, int i0, int i1) {
        int64_t *na = new_at_t.data() + (size_t)t * (Lhi + 2);
        for (int j = std::max(i0, 1); j < i1; ++j) {
            const uint64_t d = key[j] ^ key[j - 1];
            if (!d) {
                first[j] = (unsigned char)(Lhi + 1);  // same cell at every level
                continue;
            }
            const int hb = 63 - __builtin_clzll(d);
            first[j] = (unsigned char)(Lhi - hb / 3);
            ++na[first[j]];
        }
    });
    for (int t = 0; t < T; ++t)
        for (int l = 0; l < Lhi + 2; ++l) new_at[l] += new_at_t[(size_t)t * (Lhi + 2) + l];
    // the cells of levels 0..L with their blob ranges, parents and children, the
    // interaction lists, the adjacent leaves and the work items of leaf level L
    auto build = [&](int L, FmmPlan &q) -> int {
        // cells of every level in Morton order, with their blob ranges
        std::vector<std::vector<int>> starts(L + 1, std::vector<int>(1, 0));
        for (int j = 1; j < N; ++j)
            for (int l = first[j]; l <= L; ++l) starts[l].push_back(j);
        std::vector<int4> cc;
        std::vector<int2> rng;
        std::vector<uint64_t> pk;
        std::vector<int> lvl(L + 2, 0);
        for (int l = 0; l <= L; ++l) {
            lvl[l] = (int)cc.size();
            const int sh = 3 * (Lhi - l), dl = Lhi - l;
            const std::vector<int> &st = starts[l];
            for (size_t t = 0; t < st.size(); ++t) {
                const int j = st[t], e = t + 1 < st.size() ? st[t + 1] : N;
                const int i0 = idx[j];
                cc.push_back(make_int4(crd[3 * (size_t)i0] >> dl, crd[3 * (size_t)i0 + 1] >> dl,
                                       crd[3 * (size_t)i0 + 2] >> dl, l));
                rng.push_back(make_int2(j, e));
                pk.push_back(key[j] >> sh);
            }
        }
        lvl[L + 1] = (int)cc.size();
        const int ncell = (int)cc.size();
        std::vector<int> parent(ncell, -1);
        std::vector<int2> kids(ncell, make_int2(0, 0));
        for (int l = 1; l <= L; ++l) {
            int p = lvl[l - 1];
            for (int c = lvl[l]; c < lvl[l + 1]; ++c) {
                while (rng[p].y <= rng[c].x) ++p;
                parent[c] = p;
                if (kids[p].y == 0) kids[p] = make_int2(c, c + 1);
                else kids[p].y = c + 1;
            }
        }
        std::vector<CellHash> hash(L + 1);
        for (int l = 0; l <= L; ++l)
            hash[l].build(pk.data() + lvl[l], lvl[l + 1] - lvl[l], lvl[l], T);
        auto find = [&](int l, int x, int y, int z) -> int { return hash[l].get(l, x, y, z); };
        auto adjacent = [&](int c1, int c2) {
            return std::abs(cc[c1].x - cc[c2].x) <= 1 && std::abs(cc[c1].y - cc[c2].y) <= 1 &&
                   std::abs(cc[c1].z - cc[c2].z) <= 1;
        };
        // interaction lists (levels 2..L) and the adjacent leaves
        std::vector<int> il_ptr, il;
        lists_by_item(T, ncell, il_ptr, il, [&](int c, std::vector<int> &out) {
            const int l = cc[c].w;
            if (l < 2) return;
            const int4 pc = cc[parent[c]];
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int q = find(l - 1, pc.x + dx, pc.y + dy, pc.z + dz);
                        if (q < 0) continue;
                        for (int ch = kids[q].x; ch < kids[q].y; ++ch)
                            if (!adjacent(ch, c)) out.push_back(ch);
                    }
        });
        const int leaf0 = lvl[L], nleaf = lvl[L + 1] - lvl[L];
        std::vector<int> near_ptr, nearl;
        lists_by_item(T, nleaf, near_ptr, nearl, [&](int i, std::vector<int> &out) {
            const int4 c4 = cc[leaf0 + i];
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int q = find(L, c4.x + dx, c4.y + dy, c4.z + dz);
                        if (q >= 0) out.push_back(q);
                    }
        });
        std::vector<int2> work;
        for (int c = leaf0; c < leaf0 + nleaf; ++c)
            for (int k0 = rng[c].x; k0 < rng[c].y; k0 += kNearBlock) work.push_back(make_int2(c, k0));
        // every target sees every source exactly once: the adjacent leaves and the
        // interaction lists of its ancestors hold N blobs between them, and every
        // index handed to a kernel is in range
        for (int c = leaf0; c < leaf0 + nleaf; ++c) {
            int64_t cnt = 0;
            for (int e = near_ptr[c - leaf0]; e < near_ptr[c - leaf0 + 1]; ++e) {
                const int q = nearl[e];
                if (q < leaf0 || q >= leaf0 + nleaf) {
                    *msg = "fast product: internal error (near list)";
                    return ARB_E_ARG;
                }
                cnt += rng[q].y - rng[q].x;
            }
            for (int a2 = c; a2 >= 0 && cc[a2].w >= 2; a2 = parent[a2])
                for (int e = il_ptr[a2]; e < il_ptr[a2 + 1]; ++e) cnt += rng[il[e]].y - rng[il[e]].x;
            if (cnt != N) {
                *msg = "fast product: internal error (cells do not partition the blobs)";
                return ARB_E_ARG;
            }
        }
        q.L = L;
        q.ncell = ncell;
        q.nleaf = nleaf;
        // M2L pair evaluations: n^3 per proxy of each listed cell, or per blob
        // when the listed cell holds fewer blobs than proxies
        q.n_m2l_pairs = 0;
        for (int e = 0; e < (int)il.size(); ++e)
            q.n_m2l_pairs += (int64_t)P * std::min(P, rng[il[e]].y - rng[il[e]].x);
        q.n_near_pairs = 0;
        for (int c = leaf0; c < leaf0 + nleaf; ++c)
            for (int e = near_ptr[c - leaf0]; e < near_ptr[c - leaf0 + 1]; ++e)
                q.n_near_pairs +=
                    (int64_t)(rng[c].y - rng[c].x) * (rng[nearl[e]].y - rng[nearl[e]].x);
        q.lvl = std::move(lvl);
        q.cc = std::move(cc);
        q.rng = std::move(rng);
        q.parent = std::move(parent);
        q.kids = std::move(kids);
        q.il_ptr = std::move(il_ptr);
        q.il = std::move(il);
        q.near_ptr = std::move(near_ptr);
        q.nearl = std::move(nearl);
        q.work = std::move(work);
        return 0;
    };
    // leaf level
    int rc;
    if (Lhi < 2) {
        rc = build(0, pl);
    } else if (levels > 0) {
        rc = build(levels < 2 ? 0 : std::min(levels, Lhi), pl);
    } else if (leaf > 0) {
        // the shallowest level whose mean occupancy is at most `leaf`
        int L = Lhi;
        int64_t cells = 1;
        for (int l = 1; l <= Lhi; ++l) {
            cells += new_at[l];
            if (l >= 2 && (int64_t)N <= (int64_t)leaf * cells) {
                L = l;
                break;
            }
        }
        rc = build(L, pl);
    } else {
        // the level with the fewest pair evaluations: deeper from level 2 while
        // the count falls.  Counted level by level (the interaction lists of the
        // shallower levels are the same for every leaf level), then built once.
        // the cells of level l: each host thread finds the cell starts in its
        // slice of the sorted blobs, the slices' lists then joined in order
        // (each thread fills its own cells, at the offset of its slice; a cell's
        // coordinates are decoded from its Morton key)
        std::vector<std::vector<int>> st_t((size_t)T);
        std::vector<size_t> st_off((size_t)T + 1);
        std::vector<int> st_next((size_t)T);
        auto cells_of = [&](int l, std::vector<int4> &c4, std::vector<int2> &r2,
                            std::vector<uint64_t> &k) {
            parallel_slices(T, N, [&](int t, int i0, int i1) {
                std::vector<int> &v = st_t[t];
                v.clear();
                for (int j = i0; j < i1; ++j)
                    if (j == 0 || first[j] <= l) v.push_back(j);
            });
            st_off[0] = 0;
            for (int t = 0; t < T; ++t) st_off[t + 1] = st_off[t] + st_t[t].size();
            for (int t = T - 1, nx = N; t >= 0; --t) {  // first cell start after slice t
                st_next[t] = nx;
                if (!st_t[t].empty()) nx = st_t[t][0];
            }
            const size_t nc = st_off[T];
            c4.resize(nc);
            r2.resize(nc);
            k.resize(nc);
            const int sh = 3 * (Lhi - l);
            parallel_slices(T, T, [&](int t, int, int) {
                const std::vector<int> &v = st_t[t];
                const size_t c0 = st_off[t];
                for (size_t e = 0; e < v.size(); ++e) {
                    const uint64_t kc = key[v[e]] >> sh;
                    c4[c0 + e] = make_int4(compact3(kc >> 2), compact3(kc >> 1), compact3(kc), l);
                    r2[c0 + e] = make_int2(v[e], e + 1 < v.size() ? v[e + 1] : st_next[t]);
                    k[c0 + e] = kc;
                }
            });
        };
        std::vector<int4> pc, cc2;
        std::vector<int2> pr, rr;
        std::vector<uint64_t> pk2, kk2;
        CellHash ph, ch;
        cells_of(1, pc, pr, pk2);
        ph.build(pk2.data(), (int)pk2.size(), 0, T);
        int64_t m2l_total = 0, best = -1;
        int L = 2;
        for (int l = 2; l <= Lhi; ++l) {
            cells_of(l, cc2, rr, kk2);
            ch.build(kk2.data(), (int)kk2.size(), 0, T);
            // children of each parent (contiguous) and the parent of each cell
            std::vector<int2> kid(pc.size());
            std::vector<int> par(cc2.size());
            for (size_t p = 0, c = 0; p < pc.size(); ++p) {
                const size_t c0 = c;
                while (c < cc2.size() && rr[c].x < pr[p].y) par[c++] = (int)p;
                kid[p] = make_int2((int)c0, (int)c);
            }
            // integer counts over slices of the cells on host threads
            const int ncl = (int)cc2.size();
            const int Tc = std::max(1, std::min(T, ncl / 256));
            std::vector<int64_t> part(2 * (size_t)Tc, 0);
            parallel_slices(Tc, ncl, [&](int t, int c0, int c1) {
                int64_t m2l = 0, near = 0;
                for (int c = c0; c < c1; ++c) {
                    const int4 q = pc[par[c]];
                    int64_t adj = 0;
                    for (int dx = -1; dx <= 1; ++dx)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dz = -1; dz <= 1; ++dz) {
                                const int g = ph.get(l - 1, q.x + dx, q.y + dy, q.z + dz);
                                if (g >= 0)
                                    for (int k = kid[g].x; k < kid[g].y; ++k)
                                        if (std::abs(cc2[k].x - cc2[c].x) > 1 ||
                                            std::abs(cc2[k].y - cc2[c].y) > 1 ||
                                            std::abs(cc2[k].z - cc2[c].z) > 1)
                                            m2l += (int64_t)P * std::min(P, rr[k].y - rr[k].x);
                                const int e =
                                    ch.get(l, cc2[c].x + dx, cc2[c].y + dy, cc2[c].z + dz);
                                if (e >= 0) adj += rr[e].y - rr[e].x;
                            }
                    near += adj * (rr[c].y - rr[c].x);
                }
                part[2 * (size_t)t] = m2l;
                part[2 * (size_t)t + 1] = near;
            });
            int64_t near_pairs = 0;
            for (int t = 0; t < Tc; ++t) {
                m2l_total += part[2 * (size_t)t];
                near_pairs += part[2 * (size_t)t + 1];
            }
            const int64_t cl = near_pairs + m2l_total;
            if (best >= 0 && cl >= best) break;
            best = cl;
            L = l;
            pc.swap(cc2);
            pr.swap(rr);
            pk2.swap(kk2);
            std::swap(ph, ch);
        }
        rc = build(L, pl);
    }
    if (rc) return rc;
    // Chebyshev points, Lagrange denominators, parent polynomials at child proxies
    std::vector<float> tab(kTabSize, 0.f);
    double xn[kFmmMaxOrder];
    for (int k = 0; k < n; ++k) xn[k] = std::cos((2 * k + 1) * kPi / (2 * n));
    for (int k = 0; k < n; ++k) {
        double den = 1.0;
        for (int j = 0; j < n; ++j)
            if (j != k) den *= xn[k] - xn[j];
        tab[kTabNode + k] = (float)xn[k];
        tab[kTabDen + k] = (float)(1.0 / den);
    }
    for (int sg = 0; sg < 2; ++sg)
        for (int k = 0; k < n; ++k)
            for (int m = 0; m < n; ++m) {
                const double u = (sg ? 0.5 : -0.5) + 0.5 * xn[m];
                double p = 1.0;
                for (int j = 0; j < n; ++j)
                    if (j != k) p *= (u - xn[j]) / (xn[k] - xn[j]);
                tab[kTabT1 + (sg * kFmmMaxOrder + k) * kFmmMaxOrder + m] = (float)p;
            }
    pl.n = n;
    pl.P = P;
    pl.o[0] = o[0];
    pl.o[1] = o[1];
    pl.o[2] = o[2];
    pl.S = S;
    pl.perm.assign(idx, idx + N);  // sorted position -> blob
    pl.tab = std::move(tab);
    return 0;
}

int fmm_build(FmmState &F, hipStream_t s, int N, const double *pos_dev, const float4 *hi,
              const float4 *lo, double a, int order, int levels, int leaf, int channels,
              std::string *msg) {
    F.N = 0;
    F.ready = false;
    const int n = order > 0 ? order : kFmmDefaultOrder;
    if (n < 2 || n > kFmmMaxOrder || levels < 0 || leaf < 0 || N < 0) {
        *msg = "fast product: order must be 2..8, levels and leaf >= 0";
        return ARB_E_ARG;
    }
    F.n = n;
    F.P = n * n * n;
    ++F.version;
    if (N == 0) {
        F.ready = true;
        return 0;
    }
    if (!F.host) F.host = std::make_shared<FmmHostCache>();
    FmmHostCache &hc = *F.host;
    std::vector<double> hpage;  // pageable fallback when pinned memory is refused
    double *h = hc.positions(3 * (size_t)N);
    if (!h) {
        hpage.resize(3 * (size_t)N);
        h = hpage.data();
    }
    if (hipMemcpyAsync(h, pos_dev, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        *msg = "fast product: copying positions failed";
        return ARB_E_DEVICE;
    }
    FmmPlan &pl = hc.plan;
    const int prc = fmm_plan(pl, hc.scratch, N, h, a, n, levels, leaf, msg);
    if (prc) return prc;
    // upload
    const int P = F.P, ncell = pl.ncell;
    auto up = [&](DevBuf &b, const void *src, size_t bytes) -> bool {
        if (b.ensure(std::max<size_t>(bytes, 16)) != hipSuccess) return false;
        return bytes == 0 ||
               hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    };
    bool ok = up(F.perm, pl.perm.data(), pl.perm.size() * sizeof(int)) &&
              up(F.cc, pl.cc.data(), pl.cc.size() * sizeof(int4)) &&
              up(F.rng, pl.rng.data(), pl.rng.size() * sizeof(int2)) &&
              up(F.parent, pl.parent.data(), pl.parent.size() * sizeof(int)) &&
              up(F.kids, pl.kids.data(), pl.kids.size() * sizeof(int2)) &&
              up(F.il_ptr, pl.il_ptr.data(), pl.il_ptr.size() * sizeof(int)) &&
              up(F.il, pl.il.data(), pl.il.size() * sizeof(int)) &&
              up(F.near_ptr, pl.near_ptr.data(), pl.near_ptr.size() * sizeof(int)) &&
              up(F.nearl, pl.nearl.data(), pl.nearl.size() * sizeof(int)) &&
              up(F.work, pl.work.data(), pl.work.size() * sizeof(int2)) &&
              up(F.tab, pl.tab.data(), pl.tab.size() * sizeof(float)) &&
              F.shi.ensure((size_t)N * sizeof(float4)) == hipSuccess &&
              F.slo.ensure((size_t)N * sizeof(float4)) == hipSuccess &&
              F.slam.ensure((size_t)N * sizeof(double4)) == hipSuccess &&
              F.qhat.ensure((size_t)ncell * P * sizeof(double4)) == hipSuccess &&
              F.v.ensure((size_t)ncell * P * 3 * sizeof(double)) == hipSuccess &&
              (channels < 2 ||
               (F.slam2.ensure((size_t)N * sizeof(double4)) == hipSuccess &&
                F.qhat2.ensure((size_t)ncell * P * sizeof(double4)) == hipSuccess &&
                F.v2.ensure((size_t)ncell * P * 3 * sizeof(double)) == hipSuccess));
    const int nc_m2l = pl.L >= 2 ? pl.lvl[pl.L + 1] - pl.lvl[2] : 0;
    const int splits = nc_m2l > 0 ? m2l_splits(nc_m2l) : 1;
    ok = ok && (splits == 1 ||
                F.vsplit.ensure((size_t)nc_m2l * splits * P * 3 * channels * sizeof(double)) ==
                    hipSuccess);
    if (!ok) {
        *msg = "fast product: device allocation or copy failed";
        return ARB_E_DEVICE;
    }
    fmm_sort_pos_kernel<<<(N + 255) / 256, 256, 0, s>>>(N, F.perm.as<int>(), hi, lo,
                                                         F.shi.as<float4>(), F.slo.as<float4>());
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        *msg = "fast product: device error while sorting positions";
        return ARB_E_DEVICE;
    }
    F.L = pl.L;
    F.lvl = pl.lvl;
    F.splits = splits;
    F.o[0] = pl.o[0] / a;
    F.o[1] = pl.o[1] / a;
    F.o[2] = pl.o[2] / a;
    F.S = pl.S / a;
    F.ncell = pl.ncell;
    F.nleaf = pl.nleaf;
    F.nwork = (int)pl.work.size();
    F.n_il = (int64_t)pl.il.size();
    F.n_m2l_pairs = pl.n_m2l_pairs;
    F.n_near_pairs = pl.n_near_pairs;
    F.channels = channels;
    F.N = N;
    F.ready = true;
    return 0;
}

namespace {

template <bool WALL, class A>
void fmm_run(const FmmState &F, hipStream_t s, const double *lam, double *partial) {
    const int N = F.N, L = F.L, P = F.P;
    const Geo g{F.o[0], F.o[1], F.o[2], F.S, F.n, P};
    const int B = round_up(P, kWave);
    const float *tab = F.tab.as<float>();
    Vec4<A> *slam = F.slam.as<Vec4<A>>(), *qhat = F.qhat.as<Vec4<A>>();
    fmm_gather_lam_kernel<A><<<(N + 255) / 256, 256, 0, s>>>(N, F.perm.as<int>(), lam, slam);
    if (L >= 2) {
        fmm_p2m_kernel<A><<<F.lvl[L + 1] - F.lvl[L], B, 0, s>>>(
            g, tab, F.cc.as<int4>(), F.rng.as<int2>(), F.lvl[L], F.shi.as<float4>(),
            F.slo.as<float4>(), slam, qhat);
        with_order(F.n, [&](auto o) {
            for (int l = L - 1; l >= 2; --l)
                fmm_m2m_kernel<A, decltype(o)::value><<<F.lvl[l + 1] - F.lvl[l], B, 0, s>>>(
                    g, tab, F.cc.as<int4>(), F.kids.as<int2>(), F.lvl[l], qhat);
        });
        const int groups = m2l_groups(P);
        const size_t lds = (size_t)groups * P * (sizeof(Vec4<A>) + sizeof(float4)) +
                           (size_t)3 * (groups - 1) * P * sizeof(double) +
                           kTabSize * sizeof(float);
        const int nc = F.lvl[L + 1] - F.lvl[2], splits = F.splits;
        fmm_m2l_kernel<WALL, A><<<round_up(nc * splits, 8 * kXcdChunk), round_up(groups * P, kWave),
                                  lds, s>>>(
            g, tab, F.cc.as<int4>(), F.il_ptr.as<int>(), F.il.as<int>(), F.lvl[2], nc * splits,
            groups, splits,
            F.rng.as<int2>(), F.shi.as<float4>(), F.slo.as<float4>(), slam, qhat,
            F.v.as<double>(), F.vsplit.as<double>());
        if (splits > 1) {
            const int64_t m = (int64_t)nc * P * 3;
            fmm_split_sum_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
                m, splits, P * 3, F.vsplit.as<double>(), F.v.as<double>() + (size_t)F.lvl[2] * P * 3);
        }
        with_order(F.n, [&](auto o) {
            for (int l = 3; l <= L; ++l)
                fmm_l2l_kernel<decltype(o)::value><<<F.lvl[l + 1] - F.lvl[l], B, 0, s>>>(
                    g, tab, F.cc.as<int4>(), F.parent.as<int>(), F.lvl[l], F.v.as<double>());
        });
    }
    fmm_near_kernel<WALL, A><<<round_up(F.nwork, 8 * kXcdChunk), kNearBlock, 0, s>>>(
        g, tab, N, L >= 2 ? 1 : 0, F.cc.as<int4>(), F.rng.as<int2>(), F.near_ptr.as<int>(),
        F.nearl.as<int>(), F.lvl[L], F.work.as<int2>(), F.nwork, F.perm.as<int>(),
        F.shi.as<float4>(),
        F.slo.as<float4>(), slam, F.v.as<double>(), partial);
}

}  // namespace

void fmm_apply(const FmmState &F, hipStream_t s, bool wall, bool fp64, const double *lam,
               double *partial) {
    if (F.N == 0) return;
    if (wall)
        fp64 ? fmm_run<true, double>(F, s, lam, partial) : fmm_run<true, float>(F, s, lam, partial);
    else
        fp64 ? fmm_run<false, double>(F, s, lam, partial)
             : fmm_run<false, float>(F, s, lam, partial);
}

}  // namespace arb

namespace arb {

namespace {

template <class A>
void fmm_run6(const FmmState &F, hipStream_t s, const double *x6, double inv_a, double *partial) {
    const int M = F.N, L = F.L, P = F.P;
    const Geo g{F.o[0], F.o[1], F.o[2], F.S, F.n, P};
    const int B = round_up(P, kWave);
    const float *tab = F.tab.as<float>();
    Vec4<A> *sf = F.slam.as<Vec4<A>>(), *st = F.slam2.as<Vec4<A>>();
    Vec4<A> *qf = F.qhat.as<Vec4<A>>(), *qt = F.qhat2.as<Vec4<A>>();
    double *vu = F.v.as<double>(), *vw = F.v2.as<double>();
    fmm_gather6_kernel<A><<<(M + 255) / 256, 256, 0, s>>>(M, F.perm.as<int>(), x6, inv_a, sf, st);
    if (L >= 2) {
        const int nl = F.lvl[L + 1] - F.lvl[L];
        for (int ch = 0; ch < 2; ++ch)
            fmm_p2m_kernel<A><<<nl, B, 0, s>>>(g, tab, F.cc.as<int4>(), F.rng.as<int2>(),
                                               F.lvl[L], F.shi.as<float4>(), F.slo.as<float4>(),
                                               ch ? st : sf, ch ? qt : qf);
        with_order(F.n, [&](auto o) {
            for (int l = L - 1; l >= 2; --l)
                for (int ch = 0; ch < 2; ++ch)
                    fmm_m2m_kernel<A, decltype(o)::value><<<F.lvl[l + 1] - F.lvl[l], B, 0, s>>>(
                        g, tab, F.cc.as<int4>(), F.kids.as<int2>(), F.lvl[l], ch ? qt : qf);
        });
        const int groups = m2l_groups(P);
        const size_t lds = (size_t)groups * P * (2 * sizeof(Vec4<A>) + sizeof(float4)) +
                           (size_t)6 * (groups - 1) * P * sizeof(double) +
                           kTabSize * sizeof(float);
        const int nc = F.lvl[L + 1] - F.lvl[2], splits = F.splits;
        fmm_m2l6_kernel<A><<<round_up(nc * splits, 8 * kXcdChunk), round_up(groups * P, kWave), lds,
                             s>>>(
            g, tab, F.cc.as<int4>(), F.il_ptr.as<int>(), F.il.as<int>(), F.lvl[2], nc * splits,
            groups, splits,
            F.rng.as<int2>(), F.shi.as<float4>(), F.slo.as<float4>(), sf, st, qf, qt, vu, vw,
            F.vsplit.as<double>());
        if (splits > 1) {
            const int64_t m = (int64_t)nc * P * 3;
            for (int ch = 0; ch < 2; ++ch)
                fmm_split_sum_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
                    m, splits, P * 3, F.vsplit.as<double>() + ch * (size_t)nc * splits * P * 3,
                    (ch ? vw : vu) + (size_t)F.lvl[2] * P * 3);
        }
        with_order(F.n, [&](auto o) {
            for (int l = 3; l <= L; ++l)
                for (int ch = 0; ch < 2; ++ch)
                    fmm_l2l_kernel<decltype(o)::value><<<F.lvl[l + 1] - F.lvl[l], B, 0, s>>>(
                        g, tab, F.cc.as<int4>(), F.parent.as<int>(), F.lvl[l], ch ? vw : vu);
        });
    }
    fmm_near6_kernel<A><<<round_up(F.nwork, 8 * kXcdChunk), kNearBlock, 0, s>>>(
        g, tab, M, L >= 2 ? 1 : 0, F.cc.as<int4>(), F.rng.as<int2>(), F.near_ptr.as<int>(),
        F.nearl.as<int>(), F.lvl[L], F.work.as<int2>(), F.nwork, F.perm.as<int>(),
        F.shi.as<float4>(),
        F.slo.as<float4>(), sf, st, vu, vw, partial);
}

}  // namespace

void fmm_apply6(const FmmState &F, hipStream_t s, bool fp64, const double *x6, double inv_a,
                double *partial) {
    if (F.N == 0) return;
    fp64 ? fmm_run6<double>(F, s, x6, inv_a, partial) : fmm_run6<float>(F, s, x6, inv_a, partial);
}

}  // namespace arb

int arb_fmm_plan(int N, const double *pos, double a, int order, int levels, int leaf,
                 arb_fmm_stats *out) {
    using namespace arb;
    if (N < 0 || (N > 0 && !pos) || !(a > 0.0) || !out ||
        (order != 0 && (order < 2 || order > kFmmMaxOrder)) || levels < 0 ||
        levels > kFmmMaxLevel || leaf < 0)
        return ARB_E_ARG;
    const int n = order > 0 ? order : kFmmDefaultOrder;
    *out = arb_fmm_stats{};
    out->order = n;
    if (N == 0) return ARB_OK;
    const auto t0 = std::chrono::steady_clock::now();
    // one scratch kept for the process (plans on several threads at once: the
    // others take scratch of their own for the call)
    static std::mutex mu;
    static PlanScratch kept;
    FmmPlan pl;
    int rc = 0;
    try {
        std::string msg;
        std::unique_lock<std::mutex> lk(mu, std::try_to_lock);
        if (lk.owns_lock()) {
            rc = fmm_plan(pl, kept, N, pos, a, n, levels, leaf, &msg);
        } else {
            PlanScratch own;
            rc = fmm_plan(pl, own, N, pos, a, n, levels, leaf, &msg);
        }
    } catch (...) {  // host allocation or worker-thread failure: no exception crosses the ABI
        return ARB_E_HOST;
    }
    if (rc) return rc;
    out->levels = pl.L;
    out->cells = pl.ncell;
    out->leaves = pl.nleaf;
    out->near_pairs = pl.n_near_pairs;
    out->interactions = (long long)pl.il.size();
    out->m2l_pairs = pl.n_m2l_pairs;
    out->build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    uint64_t h = 0xcbf29ce484222325ull;
    fnv1a(h, pl.perm);
    fnv1a(h, pl.lvl);
    fnv1a(h, pl.parent);
    fnv1a(h, pl.il_ptr);
    fnv1a(h, pl.il);
    fnv1a(h, pl.near_ptr);
    fnv1a(h, pl.nearl);
    fnv1a(h, pl.cc);
    fnv1a(h, pl.rng);
    fnv1a(h, pl.kids);
    fnv1a(h, pl.work);
    fnv1a(h, pl.tab);
    out->plan_hash = (unsigned long long)h;
    return ARB_OK;
}
