// Rigid-body kinematics and constraints on gfx950 (Sec. 2.1-2.3, App. A, App. B).
//
//  rotations       R = 2 [p p^T + s p^x + (s^2 - 1/2) I] per body (App. B, Eq. rot_mat)
//  blob_geometry   r_i = q_p + R_p r_i^ref and d_i = r_i - q_p (Sec. 2.3)
//  K_apply         (K U)_i = u_p + w_p x d_i (Eq. no-slip)
//  KT_CT_apply     sign*(K^T lambda)_p + (C^T phi)_p: one wavefront per body,
//                  lanes stride over its blobs, shuffle reduction (Eq. balance)
//  constraint_rows lab-frame row coefficients of C and B (Eq. dg, App. A)
//  C_apply         (C U)_k
//  euler_update    q += dt u, theta <- theta_{w dt} . theta (Sec. 2.1, Sec. 4.3)
#include "common.h"

namespace arb {

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

__device__ __forceinline__ void matvec3(const double *R, const double *v, double *o) {
    o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ void rotations_kernel(int M, const double *__restrict__ theta, double *__restrict__ R9) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    double R[9];
    rotation_from_quat(theta + 4 * (size_t)p, R);
    for (int k = 0; k < 9; ++k) R9[9 * (size_t)p + k] = R[k];
}

__global__ void geometry_kernel(int N, const int *__restrict__ bob, const double *__restrict__ q,
                                const double *__restrict__ R9, const double *__restrict__ r_ref,
                                double *__restrict__ pos, double *__restrict__ dvec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int p = bob[i];
    double d[3];
    matvec3(R9 + 9 * (size_t)p, r_ref + 3 * (size_t)i, d);
    for (int c = 0; c < 3; ++c) {
        dvec[3 * (size_t)i + c] = d[c];
        pos[3 * (size_t)i + c] = q[3 * (size_t)p + c] + d[c];
    }
}

__global__ void K_kernel(int N, const int *__restrict__ bob, const double *__restrict__ dvec,
                         const double *__restrict__ U, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double *Up = U + 6 * (size_t)bob[i];
    const double *d = dvec + 3 * (size_t)i;
    double w[3] = {Up[3], Up[4], Up[5]}, c[3];
    cross3(w, d, c);
    for (int k = 0; k < 3; ++k) out[3 * (size_t)i + k] = Up[k] + c[k];
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// one wavefront per body; blockDim = 256 -> 4 bodies per block
__global__ __launch_bounds__(256) void KT_CT_kernel(
    int M, const int *__restrict__ blob_off, const double *__restrict__ dvec,
    const double *__restrict__ lam, double sign, const int *__restrict__ brow_ptr,
    const int *__restrict__ brow_ent, const double *__restrict__ crow,
    const double *__restrict__ phi, double *__restrict__ out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int p = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (p >= M) return;  // whole wavefront exits together
    double f[6] = {0, 0, 0, 0, 0, 0};
    if (lam) {
        for (int i = blob_off[p] + lane; i < blob_off[p + 1]; i += kWave) {
            const double l0 = lam[3 * (size_t)i], l1 = lam[3 * (size_t)i + 1],
                         l2 = lam[3 * (size_t)i + 2];
            const double d0 = dvec[3 * (size_t)i], d1 = dvec[3 * (size_t)i + 1],
                         d2 = dvec[3 * (size_t)i + 2];
            f[0] += l0;
            f[1] += l1;
            f[2] += l2;
            f[3] += d1 * l2 - d2 * l1;
            f[4] += d2 * l0 - d0 * l2;
            f[5] += d0 * l1 - d1 * l0;
        }
    }
    for (int k = 0; k < 6; ++k) f[k] = sign * wave_sum(f[k]);
    if (lane == 0) {
        if (phi) {
            for (int e = brow_ptr[p]; e < brow_ptr[p + 1]; ++e) {
                const int ent = brow_ent[e];
                const int row = ent >> 1, side = ent & 1;
                const double *c = crow + 12 * (size_t)row + 6 * side;
                const double ph = phi[row];
                for (int k = 0; k < 6; ++k) f[k] += ph * c[k];
            }
        }
        for (int k = 0; k < 6; ++k) out[6 * (size_t)p + k] = f[k];
    }
}

// row kinds: 0 = projected link row, 1 = general row
__global__ void constraint_rows_kernel(int Nc, const int *__restrict__ row_p,
                                       const int *__restrict__ row_q,
                                       const int *__restrict__ row_kind,
                                       const int *__restrict__ row_src,
                                       const int *__restrict__ row_m,
                                       const double *__restrict__ R9,
                                       const double *__restrict__ dl_p,
                                       const double *__restrict__ dl_q,
                                       const double *__restrict__ dldot_p,
                                       const double *__restrict__ dldot_q,
                                       const double *__restrict__ proj,
                                       const double *__restrict__ gcoef,
                                       const double *__restrict__ grhs,
                                       double *__restrict__ crow, double *__restrict__ B) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Nc) return;
    const int p = row_p[k], q = row_q[k], src = row_src[k];
    const double *Rp = R9 + 9 * (size_t)p;
    double c[12];
    double b;
    if (row_kind[k] == 0) {
        double d[3], lp[3], lq[3] = {0, 0, 0}, Bn[3], t[3];
        matvec3(Rp, proj + 9 * (size_t)src + 3 * row_m[k], d);
        matvec3(Rp, dl_p + 3 * (size_t)src, lp);
        matvec3(Rp, dldot_p + 3 * (size_t)src, t);
        for (int a = 0; a < 3; ++a) Bn[a] = -t[a];
        if (q >= 0) {
            const double *Rq = R9 + 9 * (size_t)q;
            matvec3(Rq, dl_q + 3 * (size_t)src, lq);
            matvec3(Rq, dldot_q + 3 * (size_t)src, t);
        } else {
            for (int a = 0; a < 3; ++a) t[a] = dldot_q[3 * (size_t)src + a];
        }
        for (int a = 0; a < 3; ++a) Bn[a] += t[a];
        double lpd[3], lqd[3];
        cross3(lp, d, lpd);
        cross3(lq, d, lqd);
        for (int a = 0; a < 3; ++a) {
            c[a] = d[a];
            c[3 + a] = lpd[a];
            c[6 + a] = q >= 0 ? -d[a] : 0.0;
            c[9 + a] = q >= 0 ? -lqd[a] : 0.0;
        }
        b = d[0] * Bn[0] + d[1] * Bn[1] + d[2] * Bn[2];
    } else {
        const double *g = gcoef + 12 * (size_t)src;
        for (int blk = 0; blk < 4; ++blk) matvec3(Rp, g + 3 * blk, c + 3 * blk);
        if (q < 0)
            for (int a = 6; a < 12; ++a) c[a] = 0.0;
        b = grhs[src];
    }
    for (int a = 0; a < 12; ++a) crow[12 * (size_t)k + a] = c[a];
    B[k] = b;
}

__global__ void C_kernel(int Nc, const int *__restrict__ row_p, const int *__restrict__ row_q,
                         const double *__restrict__ crow, const double *__restrict__ U,
                         double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Nc) return;
    const double *c = crow + 12 * (size_t)k;
    const double *Up = U + 6 * (size_t)row_p[k];
    double s = 0.0;
    for (int a = 0; a < 6; ++a) s += c[a] * Up[a];
    const int q = row_q[k];
    if (q >= 0) {
        const double *Uq = U + 6 * (size_t)q;
        for (int a = 0; a < 6; ++a) s += c[6 + a] * Uq[a];
    }
    out[k] = s;
}

__global__ void euler_kernel(int M, const double *__restrict__ U, double dt, double *__restrict__ q,
                             double *__restrict__ theta) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double *Up = U + 6 * (size_t)p;
    for (int k = 0; k < 3; ++k) q[3 * (size_t)p + k] += dt * Up[k];
    // finite-rotation quaternion of gamma = w dt: [cos(g/2), sin(g/2) gamma/g]
    const double g0 = dt * Up[3], g1 = dt * Up[4], g2 = dt * Up[5];
    const double g = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    const double s2 = cos(0.5 * g);
    const double f = g > 0.0 ? sin(0.5 * g) / g : 0.5;
    const double a0 = s2, a1 = f * g0, a2 = f * g1, a3 = f * g2;
    double *t = theta + 4 * (size_t)p;
    const double b0 = t[0], b1 = t[1], b2 = t[2], b3 = t[3];
    // theta_gamma . theta (Eq. quaternion_mult)
    t[0] = a0 * b0 - (a1 * b1 + a2 * b2 + a3 * b3);
    t[1] = a0 * b1 + b0 * a1 + (a2 * b3 - a3 * b2);
    t[2] = a0 * b2 + b0 * a2 + (a3 * b1 - a1 * b3);
    t[3] = a0 * b3 + b0 * a3 + (a1 * b2 - a2 * b1);
}

void rotations(hipStream_t s, int M, const double *theta, double *R9) {
    if (M > 0) rotations_kernel<<<nblk(M, 256), 256, 0, s>>>(M, theta, R9);
}
void blob_geometry(hipStream_t s, int N, const int *bob, const double *q, const double *R9,
                   const double *r_ref, double *pos, double *dvec) {
    if (N > 0) geometry_kernel<<<nblk(N, 256), 256, 0, s>>>(N, bob, q, R9, r_ref, pos, dvec);
}
void K_apply(hipStream_t s, int N, const int *bob, const double *dvec, const double *U,
             double *out) {
    if (N > 0) K_kernel<<<nblk(N, 256), 256, 0, s>>>(N, bob, dvec, U, out);
}
void KT_CT_apply(hipStream_t s, int M, const int *blob_off, const double *dvec,
                 const double *lam, double sign, const int *brow_ptr, const int *brow_ent,
                 const double *crow, const double *phi, double *out) {
    if (M > 0)
        KT_CT_kernel<<<nblk(M, 4), 256, 0, s>>>(M, blob_off, dvec, lam, sign, brow_ptr, brow_ent,
                                                crow, phi, out);
}
void constraint_rows(hipStream_t s, int Nc, const int *row_p, const int *row_q,
                     const int *row_kind, const int *row_src, const int *row_m,
                     const double *R9, const double *dl_p, const double *dl_q,
                     const double *dldot_p, const double *dldot_q, const double *proj,
                     const double *gcoef, const double *grhs, double *crow, double *B) {
    if (Nc > 0)
        constraint_rows_kernel<<<nblk(Nc, 256), 256, 0, s>>>(Nc, row_p, row_q, row_kind, row_src,
                                                             row_m, R9, dl_p, dl_q, dldot_p,
                                                             dldot_q, proj, gcoef, grhs, crow, B);
}
void C_apply(hipStream_t s, int Nc, const int *row_p, const int *row_q, const double *crow,
             const double *U, double *out) {
    if (Nc > 0) C_kernel<<<nblk(Nc, 256), 256, 0, s>>>(Nc, row_p, row_q, crow, U, out);
}
void euler_update(hipStream_t s, int M, const double *U, double dt, double *q, double *theta) {
    if (M > 0) euler_kernel<<<nblk(M, 256), 256, 0, s>>>(M, U, dt, q, theta);
}

}  // namespace arb
