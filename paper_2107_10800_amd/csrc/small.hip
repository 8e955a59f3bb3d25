// One restart cycle of right-preconditioned GMRES (Sec. 3.1) for a small
// multiblob system in one workgroup: every Arnoldi step -- the block
// preconditioner apply (Sec. 3.1 Eq. precond), the saddle-system product of
// Sec. 2.3 Eq. linear_system with FP64 pair sums (Eq. RPY), classical
// Gram-Schmidt twice and the Givens update -- runs inside one launch, phases
// separated by workgroup barriers, and the stopping test on the residual
// estimate is taken on the device.  A system of a few hundred unknowns then
// costs a few microseconds per step instead of ten launches and a host
// round trip.  The arithmetic is that of the per-step kernels with other
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

// the Givens update of the new Hessenberg column (as arnoldi_post_dev in krylov.hip)
__device__ void givens_column(int j, int m, const double *h1, const double *h2, double hn2,
                              double *Hbar, double *cs, double *sn, double *g, double *out) {
    double *col = Hbar + (int64_t)j * (m + 1);
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

template <bool WALL>
__global__ __launch_bounds__(kThreads) void gmres_small_cycle_kernel(
    SmallSystem S, int m, int budget, double target, double *__restrict__ V,
    double *__restrict__ Hbar, double *__restrict__ cs,
    double *__restrict__ sn, double *__restrict__ g, double *__restrict__ steps) {
    // v_j, z = P^-1 v_j and w = A z in LDS (the basis V stays in memory); U^ too
    __shared__ double vs[kSmallArnoldi], zs[kSmallArnoldi], ws[kSmallArnoldi];
    __shared__ double us[6 * kSmallCycleN];
    __shared__ double hs[2][kMaxRestart + 1];
    __shared__ double red[kWaves];
    __shared__ double hn_est[2];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t n = S.n;
    const CoefD coef = make_coef<CoefD, double>(S.a);
    const size_t o_u = 3 * (size_t)S.N, o_phi = o_u + 6 * (size_t)S.M;
    int k = 0;
    for (int t = tid; t < n; t += kThreads) vs[t] = V[t];
    __syncthreads();
    for (int j = 0; j < budget; ++j) {
        const double *r = vs;
        double *z = zs;
        // ---- z = P^-1 v_j: body blocks (one wavefront per body) -------------------
        for (int p = wave; p < S.M; p += kWaves) {
            const int b0 = S.blob_off[p], mm = 3 * (S.blob_off[p + 1] - b0);
            const double *Mi = S.minv + S.mat_off[p];
            const double *Zp = S.Z + S.z_off[p];
            const double *rl = r + 3 * (size_t)b0;
            double acc[6] = {0, 0, 0, 0, 0, 0};
            for (int i = lane; i < mm; i += kWave) {
                double s = 0.0;  // M_pp^-1 is symmetric: column i, consecutive lanes
                for (int kk = 0; kk < mm; ++kk) s += Mi[(size_t)kk * mm + i] * rl[kk];
                z[3 * (size_t)b0 + i] = s;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] += Zp[(size_t)i * 6 + c] * rl[i];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] = wsum(acc[c]) + r[o_u + 6 * (size_t)p + c];
            if (lane < 6) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) s += S.Nt[36 * (size_t)p + lane * 6 + c] * acc[c];
                us[6 * p + lane] = -s;
            }
        }
        __syncthreads();
        // assemblies (one wavefront each, at most one row per lane): phi = G~ (r_phi - C U^)
        for (int a = wave; a < S.A; a += kWaves) {
            const int r0 = S.asm_row_ptr[a], na = S.asm_row_ptr[a + 1] - r0;
            double y = 0.0;
            int rk = 0;
            if (lane < na) {
                rk = S.asm_rows[r0 + lane];
                const double *c = S.crow + 12 * (size_t)rk;
                const double *Up = us + 6 * S.row_p[rk];
                double s = 0.0;
                for (int u = 0; u < 6; ++u) s += c[u] * Up[u];
                const int q = S.row_q[rk];
                if (q >= 0)
                    for (int u = 0; u < 6; ++u) s += c[6 + u] * us[6 * q + u];
                y = r[o_phi + rk] - s;
            }
            const double *Ga = S.G + S.asm_mat_off[a];
            double phi = 0.0;
            for (int l = 0; l < na; ++l) {
                const double yl = __shfl(y, l);
                if (lane < na) phi += Ga[(size_t)lane * na + l] * yl;
            }
            if (lane < na) z[o_phi + rk] = phi;
        }
        __syncthreads();
        // bodies again: U = U^ + N~ C^T phi, lambda += Z U
        for (int p = wave; p < S.M; p += kWaves) {
            double f[6] = {0, 0, 0, 0, 0, 0};
            if (S.Nc > 0)
                for (int e = S.brow_ptr[p] + lane; e < S.brow_ptr[p + 1]; e += kWave) {
                    const int ent = S.brow_ent[e], row = ent >> 1, side = ent & 1;
                    const double ph = z[o_phi + row];
#pragma unroll
                    for (int c = 0; c < 6; ++c) f[c] += ph * S.crow[12 * (size_t)row + 6 * side + c];
                }
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] = wsum(f[c]);
            double U[6];
#pragma unroll
            for (int c1 = 0; c1 < 6; ++c1) {
                double s = us[6 * p + c1];
#pragma unroll
                for (int c2 = 0; c2 < 6; ++c2) s += S.Nt[36 * (size_t)p + 6 * c1 + c2] * f[c2];
                U[c1] = s;
            }
#pragma unroll
            for (int c = 0; c < 6; ++c)
                if (lane == c) z[o_u + 6 * (size_t)p + c] = U[c];
            const int b0 = S.blob_off[p], mm = 3 * (S.blob_off[p + 1] - b0);
            const double *Zp = S.Z + S.z_off[p];
            for (int i = lane; i < mm; i += kWave) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) s += Zp[(size_t)i * 6 + c] * U[c];
                z[3 * (size_t)b0 + i] += s;
            }
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
        // body rows: -K^T lambda + C^T phi (one wavefront per body)
        for (int p = wave; p < S.M; p += kWaves) {
            double f[6] = {0, 0, 0, 0, 0, 0};
            for (int ib = S.blob_off[p] + lane; ib < S.blob_off[p + 1]; ib += kWave) {
                const double l0 = z[3 * (size_t)ib], l1 = z[3 * (size_t)ib + 1],
                             l2 = z[3 * (size_t)ib + 2];
                const double d0 = S.dvec[3 * (size_t)ib], d1 = S.dvec[3 * (size_t)ib + 1],
                             d2 = S.dvec[3 * (size_t)ib + 2];
                f[0] += l0;
                f[1] += l1;
                f[2] += l2;
                f[3] += d1 * l2 - d2 * l1;
                f[4] += d2 * l0 - d0 * l2;
                f[5] += d0 * l1 - d1 * l0;
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) f[c] = -wsum(f[c]);
            if (lane == 0) {
                if (S.Nc > 0)
                    for (int e = S.brow_ptr[p]; e < S.brow_ptr[p + 1]; ++e) {
                        const int ent = S.brow_ent[e], row = ent >> 1, side = ent & 1;
                        const double *c = S.crow + 12 * (size_t)row + 6 * side;
                        const double ph = z[o_phi + row];
                        for (int c6 = 0; c6 < 6; ++c6) f[c6] += ph * c[c6];
                    }
                for (int c = 0; c < 6; ++c) ws[o_u + 6 * (size_t)p + c] = f[c];
            }
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
            givens_column(j, m, hs[0], hs[1], hn2, Hbar, cs, sn, g, steps + 2 * j);
            hn_est[0] = steps[2 * j];
            hn_est[1] = steps[2 * j + 1];
        }
        __syncthreads();
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
    if (tid == 0) steps[2 * m] = (double)k;
}

}  // namespace

void gmres_small_cycle(hipStream_t s, const SmallSystem &S, int m, int budget, double target,
                       double *V, double *Hbar, double *cs, double *sn, double *g, double *steps) {
    if (S.wall)
        gmres_small_cycle_kernel<true>
            <<<1, kThreads, 0, s>>>(S, m, budget, target, V, Hbar, cs, sn, g, steps);
    else
        gmres_small_cycle_kernel<false>
            <<<1, kThreads, 0, s>>>(S, m, budget, target, V, Hbar, cs, sn, g, steps);
}

}  // namespace arb
