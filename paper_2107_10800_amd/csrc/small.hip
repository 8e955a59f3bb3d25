// One restart cycle of right-preconditioned GMRES (Sec. 3.1) for a small
// multiblob system in one workgroup: every Arnoldi step -- the block
// preconditioner apply (Sec. 3.1 Eq. precond), the saddle-system product of
// Sec. 2.3 Eq. linear_system with FP64 pair sums (Eq. RPY), classical
// Gram-Schmidt twice and the Givens update -- runs inside one launch, phases
// separated by workgroup barriers, and the stopping test on the residual
// estimate is taken on the device.  A system of a few hundred unknowns then
// costs a few microseconds per step instead of ten launches and a host
// round trip; the data a step reads sit in LDS (a step is a chain of short
// phases, each of which would otherwise wait on memory).  The arithmetic is that of the per-step kernels with other
// summation orders.
#include "common.h"
#include "rpy_device.h"

namespace arb {

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / kWave;

__device__ __forceinline__ double wsum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// the Givens update of the new Hessenberg column (as arnoldi_post_dev in krylov.hip),
// on LDS copies of the column, the rotations and g
__device__ void givens_column(int j, const double *h1, const double *h2, double hn2, double *col,
                              double *cs, double *sn, double *g, double *out) {
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    const double hn = sqrt(hn2);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
    }
    const double rho = hypot(col[j], col[j + 1]);
    cs[j] = col[j] / rho;
    sn[j] = col[j + 1] / rho;
    col[j] = rho;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    out[0] = hn;
    out[1] = fabs(g[j + 1]);
}

template <class T>
__device__ __forceinline__ T *stage(const T *src, size_t cnt, T *dst) {
    for (size_t t = threadIdx.x; t < cnt; t += kThreads) dst[t] = src[t];
    return dst;
}

// Everything a step reads is staged once in the dynamic LDS arena (small_layout):
// the state (positions, d_i), the preconditioner (M_pp^-1, Z_p, N~_p, G~_a),
// the constraint rows and the index arrays; v_j, z = P^-1 v_j, w = A z and U^
// live there too.  Only the Krylov basis V (written once per step, read by the
// Gram-Schmidt passes) and the Hessenberg data stay in memory.
template <bool WALL>
__global__ __launch_bounds__(kThreads) void gmres_small_cycle_kernel(
    SmallSystem Sg, int m, int budget, double target, double *__restrict__ V,
    double *__restrict__ Hbar, double *__restrict__ cs,
    double *__restrict__ sn, double *__restrict__ g, double *__restrict__ steps) {
    extern __shared__ double arena[];
    __shared__ double hs[2][kMaxRestart + 1];
    __shared__ double col[kMaxRestart + 2], cs_s[kMaxRestart + 1], sn_s[kMaxRestart + 1],
        g_s[kMaxRestart + 2];
    __shared__ double red[kWaves];
    __shared__ double hn_est[2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const SmallLayout L = small_layout(Sg);
    int *ia = reinterpret_cast<int *>(arena + L.ints);
    SmallSystem S = Sg;
    S.p64 = stage(Sg.p64, Sg.N, reinterpret_cast<double4 *>(arena + L.p64));
    S.dvec = stage(Sg.dvec, 3 * (size_t)Sg.N, arena + L.dvec);
    S.minv = stage(Sg.minv, Sg.n_minv, arena + L.minv);
    S.Z = stage(Sg.Z, Sg.n_z, arena + L.Z);
    S.Nt = stage(Sg.Nt, 36 * (size_t)Sg.M, arena + L.Nt);
    S.G = stage(Sg.G, Sg.n_g, arena + L.G);
    S.crow = stage(Sg.crow, 12 * (size_t)Sg.Nc, arena + L.crow);
    S.mat_off = stage(Sg.mat_off, Sg.M + 1, reinterpret_cast<int64_t *>(arena + L.mat_off));
    S.z_off = stage(Sg.z_off, Sg.M + 1, reinterpret_cast<int64_t *>(arena + L.z_off));
    S.asm_mat_off =
        Sg.A > 0 ? stage(Sg.asm_mat_off, Sg.A + 1, reinterpret_cast<int64_t *>(arena + L.asm_mat_off))
                 : nullptr;
    S.bob = stage(Sg.bob, Sg.N, ia + L.bob);
    S.blob_off = stage(Sg.blob_off, Sg.M + 1, ia + L.blob_off);
    S.brow_ptr = Sg.Nc > 0 ? stage(Sg.brow_ptr, Sg.M + 1, ia + L.brow_ptr) : nullptr;
    S.brow_ent = Sg.Nc > 0 ? stage(Sg.brow_ent, Sg.n_brow_ent, ia + L.brow_ent) : nullptr;
    S.row_p = stage(Sg.row_p, Sg.Nc, ia + L.row_p);
    S.row_q = stage(Sg.row_q, Sg.Nc, ia + L.row_q);
    S.asm_row_ptr = Sg.A > 0 ? stage(Sg.asm_row_ptr, Sg.A + 1, ia + L.asm_row_ptr) : nullptr;
    S.asm_rows = Sg.A > 0 ? stage(Sg.asm_rows, Sg.Nc, ia + L.asm_rows) : nullptr;
    S.perm = Sg.perm ? stage(Sg.perm, Sg.N, ia + L.perm) : nullptr;
    double *vs = arena + L.vs, *zs = arena + L.zs, *ws = arena + L.ws, *us = arena + L.us;
    double *w6 = arena + L.w6, *yv = arena + L.yv;
    int *slot_a = ia + L.slot_a;  // assembly of each slot of asm_rows
    for (int a = tid; a < Sg.A; a += kThreads)
        for (int sl = Sg.asm_row_ptr[a]; sl < Sg.asm_row_ptr[a + 1]; ++sl) slot_a[sl] = a;
    const int64_t n = S.n;
    const CoefD coef = make_coef<CoefD, double>(S.a);
    const size_t o_u = 3 * (size_t)S.N, o_phi = o_u + 6 * (size_t)S.M;
    int k = 0;
    for (int t = tid; t < n; t += kThreads) vs[t] = V[t];
    for (int t = tid; t <= m; t += kThreads) g_s[t] = g[t];
    __syncthreads();
    for (int j = 0; j < budget; ++j) {
        const double *r = vs;
        double *z = zs;
        // ---- z = P^-1 v_j, every phase a flat loop (a thread per row, per body and
        // component, or per constraint row), no wavefront reductions -----------------
        // blob rows: M_pp^-1 r_lambda (symmetric: column i, consecutive threads)
        for (int R = tid; R < 3 * S.N; R += kThreads) {
            const int p = S.bob[R / 3], b0 = S.blob_off[p], mm = 3 * (S.blob_off[p + 1] - b0);
            const int i = R - 3 * b0;
            const double *Mi = S.minv + S.mat_off[p];
            const double *rl = r + 3 * (size_t)b0;
            double s = 0.0;
            for (int kk = 0; kk < mm; ++kk) s += Mi[(size_t)kk * mm + i] * rl[kk];
            z[R] = s;
        }
        // w6 = Z_p^T r_lambda + r_U per body and component
        for (int e = tid; e < 6 * S.M; e += kThreads) {
            const int p = e / 6, c = e - 6 * p;
            const int b0 = S.blob_off[p], mm = 3 * (S.blob_off[p + 1] - b0);
            const double *Zp = S.Z + S.z_off[p];
            double acc = r[o_u + e];
            for (int i = 0; i < mm; ++i) acc += Zp[(size_t)i * 6 + c] * r[3 * (size_t)b0 + i];
            w6[e] = acc;
        }
        __syncthreads();
        // U^ = -N~ w6
        for (int e = tid; e < 6 * S.M; e += kThreads) {
            const int p = e / 6, c = e - 6 * p;
            double s = 0.0;
#pragma unroll
            for (int c2 = 0; c2 < 6; ++c2) s += S.Nt[36 * (size_t)p + 6 * c + c2] * w6[6 * p + c2];
            us[e] = -s;
        }
        __syncthreads();
        // assemblies: y = r_phi - C U^ per row, then phi = G~ y over each assembly's rows
        for (int kr = tid; kr < S.Nc; kr += kThreads) {
            const double *c = S.crow + 12 * (size_t)kr;
            const double *Up = us + 6 * S.row_p[kr];
            double s = 0.0;
            for (int u = 0; u < 6; ++u) s += c[u] * Up[u];
            const int q = S.row_q[kr];
            if (q >= 0)
                for (int u = 0; u < 6; ++u) s += c[6 + u] * us[6 * q + u];
            yv[kr] = r[o_phi + kr] - s;
        }
        __syncthreads();
        for (int sl = tid; sl < S.Nc; sl += kThreads) {
            const int a = slot_a[sl], r0 = S.asm_row_ptr[a], na = S.asm_row_ptr[a + 1] - r0;
            const double *Ga = S.G + S.asm_mat_off[a] + (size_t)(sl - r0) * na;
            double s = 0.0;
            for (int l = 0; l < na; ++l) s += Ga[l] * yv[S.asm_rows[r0 + l]];
            z[o_phi + S.asm_rows[sl]] = s;
        }
        __syncthreads();
        // U = U^ + N~ C^T phi: f = C^T phi per body and component, then U
        for (int e = tid; e < 6 * S.M; e += kThreads) {
            const int p = e / 6, c = e - 6 * p;
            double f = 0.0;
            if (S.Nc > 0)
                for (int en = S.brow_ptr[p]; en < S.brow_ptr[p + 1]; ++en) {
                    const int ent = S.brow_ent[en], row = ent >> 1, side = ent & 1;
                    f += z[o_phi + row] * S.crow[12 * (size_t)row + 6 * side + c];
                }
            w6[e] = f;
        }
        __syncthreads();
        for (int e = tid; e < 6 * S.M; e += kThreads) {
            const int p = e / 6, c = e - 6 * p;
            double s = us[e];
#pragma unroll
            for (int c2 = 0; c2 < 6; ++c2) s += S.Nt[36 * (size_t)p + 6 * c + c2] * w6[6 * p + c2];
            z[o_u + e] = s;
        }
        __syncthreads();
        // lambda += Z U per blob row
        for (int R = tid; R < 3 * S.N; R += kThreads) {
            const int p = S.bob[R / 3], b0 = S.blob_off[p];
            const double *Zr = S.Z + S.z_off[p] + (size_t)(R - 3 * b0) * 6;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 6; ++c) s += Zr[c] * z[o_u + 6 * (size_t)p + c];
            z[R] += s;
        }
        __syncthreads();
        // ---- w = A z into LDS ------------------------------------------------------
        // blob rows: M lambda - K U; tpt threads per target, sources strided (the
        // same number of passes in every thread, so the group sums below see
        // whole groups)
        for (int base = 0; base < S.N * S.tpt; base += kThreads) {
            const int tpt = S.tpt, i = (base + tid) / tpt, sl = (base + tid) % tpt;
            double ux = 0.0, uy = 0.0, uz = 0.0;
            if (i < S.N) {
                const double4 ti = S.p64[i];
                const TargetZ<double> zsc = target_z(ti.z);
                for (int jj = sl; jj < S.N; jj += tpt) {
                    const double4 sj = S.p64[jj];
                    const size_t b = 3 * (size_t)(S.perm ? S.perm[jj] : jj);
                    const double lx = z[b], ly = z[b + 1], lz = z[b + 2];
                    const double dx = ti.x - sj.x, dy = ti.y - sj.y, dz = ti.z - sj.z;
                    const double dxy2 = fma(dx, dx, dy * dy);
                    const double r2 = fma(dz, dz, dxy2);
                    const double rinv = rsq_f64(r2);
                    if (WALL) {
                        const double Rz = ti.z + sj.z;
                        const double Ri = rsq_f64(fma(Rz, Rz, dxy2));
                        const PairCoef<double> w = wall_pair_coef<double>(
                            r2, rinv, dxy2, zsc, sj.z, sj.w, -(sj.w * sj.w), Rz, Ri, coef);
                        wall_pair_apply<double>(w, w.c, w.d, dx, dy, dz, Rz, lx, ly, lz, ux, uy,
                                                uz);
                    } else {
                        rpy_free<double>(dx, dy, dz, r2, rinv, lx, ly, lz, coef, ux, uy, uz);
                    }
                }
            }
            for (int off = tpt / 2; off > 0; off >>= 1) {
                ux += __shfl_xor(ux, off);
                uy += __shfl_xor(uy, off);
                uz += __shfl_xor(uz, off);
            }
            if (i < S.N && sl == 0) {
                const int ib = S.perm ? S.perm[i] : i;
                const double *Up = z + o_u + 6 * (size_t)S.bob[ib];
                const double d0 = S.dvec[3 * (size_t)ib], d1 = S.dvec[3 * (size_t)ib + 1],
                             d2 = S.dvec[3 * (size_t)ib + 2];
                ws[3 * ib] = ux * S.scale - (Up[0] + (Up[4] * d2 - Up[5] * d1));
                ws[3 * ib + 1] = uy * S.scale - (Up[1] + (Up[5] * d0 - Up[3] * d2));
                ws[3 * ib + 2] = uz * S.scale - (Up[2] + (Up[3] * d1 - Up[4] * d0));
            }
        }
        // body rows: -K^T lambda + C^T phi per body and component
        for (int e = tid; e < 6 * S.M; e += kThreads) {
            const int p = e / 6, c = e - 6 * p;
            double f = 0.0;
            for (int ib = S.blob_off[p]; ib < S.blob_off[p + 1]; ++ib) {
                const double *l = z + 3 * (size_t)ib;
                const double *dv = S.dvec + 3 * (size_t)ib;
                // (K^T lambda)_c: the force, or d x lambda
                f += c < 3 ? l[c]
                           : (c == 3 ? dv[1] * l[2] - dv[2] * l[1]
                                     : (c == 4 ? dv[2] * l[0] - dv[0] * l[2]
                                               : dv[0] * l[1] - dv[1] * l[0]));
            }
            f = -f;
            if (S.Nc > 0)
                for (int en = S.brow_ptr[p]; en < S.brow_ptr[p + 1]; ++en) {
                    const int ent = S.brow_ent[en], row = ent >> 1, side = ent & 1;
                    f += z[o_phi + row] * S.crow[12 * (size_t)row + 6 * side + c];
                }
            ws[o_u + e] = f;
        }
        // constraint rows: C U
        for (int kr = tid; kr < S.Nc; kr += kThreads) {
            const double *c = S.crow + 12 * (size_t)kr;
            const double *Up = z + o_u + 6 * (size_t)S.row_p[kr];
            double s = 0.0;
            for (int u = 0; u < 6; ++u) s += c[u] * Up[u];
            const int q = S.row_q[kr];
            if (q >= 0)
                for (int u = 0; u < 6; ++u) s += c[6 + u] * z[o_u + 6 * (size_t)q + u];
            ws[o_phi + kr] = s;
        }
        __syncthreads();
        // ---- classical Gram-Schmidt twice, ||w||, Givens ---------------------------
        for (int pass = 0; pass < 2; ++pass) {
            double *h = hs[pass];
            for (int i = wave; i <= j; i += kWaves) {
                const double *v = V + (int64_t)i * n;
                double sacc = 0.0;
                for (int t = lane; t < n; t += kWave) sacc += v[t] * ws[t];
                sacc = wsum(sacc);
                if (lane == 0) h[i] = sacc;
            }
            __syncthreads();
            for (int t = tid; t < n; t += kThreads) {
                double acc = 0.0;
                for (int i = 0; i <= j; ++i) acc += V[(int64_t)i * n + t] * h[i];
                ws[t] -= acc;
            }
            __syncthreads();
        }
        double sq = 0.0;
        for (int t = tid; t < n; t += kThreads) sq += ws[t] * ws[t];
        sq = wsum(sq);
        if (lane == 0) red[wave] = sq;
        __syncthreads();
        if (tid == 0) {
            double hn2 = 0.0;
            for (int q = 0; q < kWaves; ++q) hn2 += red[q];
            givens_column(j, hs[0], hs[1], hn2, col, cs_s, sn_s, g_s, hn_est);
            steps[2 * j] = hn_est[0];
            steps[2 * j + 1] = hn_est[1];
        }
        __syncthreads();
        for (int i = tid; i <= j + 1; i += kThreads) Hbar[(int64_t)j * (m + 1) + i] = col[i];
        const double hn = hn_est[0], est = hn_est[1];
        k = j + 1;
        // the same value in every thread: a uniform exit (non-finite values end the
        // cycle too; the host reports them)
        if (!(est > target) || hn == 0.0 || !(hn == hn)) break;
        if (j + 1 < budget) {
            double *vn = V + (size_t)(j + 1) * n;
            const double inv = 1.0 / hn;
            for (int t = tid; t < n; t += kThreads) {
                const double v = ws[t] * inv;
                vn[t] = v;
                vs[t] = v;
            }
        }
        __syncthreads();
    }
    // g, and the rotations, for the update after the cycle
    __syncthreads();
    for (int t = tid; t <= k; t += kThreads) g[t] = g_s[t];
    for (int t = tid; t < k; t += kThreads) {
        cs[t] = cs_s[t];
        sn[t] = sn_s[t];
    }
    if (tid == 0) steps[2 * m] = (double)k;
}

}  // namespace

hipError_t gmres_small_cycle(hipStream_t s, const SmallSystem &S, int m, int budget,
                             double target, double *V, double *Hbar, double *cs, double *sn,
                             double *g, double *steps) {
    const size_t lds = small_layout(S).bytes;
    const void *fn = S.wall ? (const void *)gmres_small_cycle_kernel<true>
                            : (const void *)gmres_small_cycle_kernel<false>;
    const hipError_t e =
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (S.wall)
        gmres_small_cycle_kernel<true>
            <<<1, kThreads, lds, s>>>(S, m, budget, target, V, Hbar, cs, sn, g, steps);
    else
        gmres_small_cycle_kernel<false>
            <<<1, kThreads, lds, s>>>(S, m, budget, target, V, Hbar, cs, sn, g, steps);
    return hipGetLastError();
}

}  // namespace arb
