// Block-diagonal preconditioner of Sec. 3.1 (Eq. precond, Eq. block_diag_const_res).
//
// Build (once per state), per body p with m = 3 n_p:
//   pc_assemble  M_pp (m x m, row-major) from the same pair code as the mat-vec
//   pc_sweep     (no body above 256 rows) M_pp^-1 by the symmetric block sweep,
//                the matrix held in registers as 16 x 16 matrix-core tiles, one
//                workgroup per body; M_pp is kept.  Larger bodies:
//   pc_potrf     M_pp = L L^T in place, blocked by 32 columns: the panel is
//                factored in LDS, the trailing lower triangle updated in 64 x 64
//                tiles on the FP64 matrix cores; the inverses of the 32 x 32
//                diagonal blocks of L are kept for the next step
//   pc_trtri     X = L^-1 by block forward substitution on the identity, one
//                workgroup per (body, 32 columns), the block column held in LDS;
//                every block step is a small GEMM on the matrix cores because
//                the diagonal blocks are applied through their stored inverses;
//                X^T is kept in the strictly upper triangle
//   pc_lauum     M_pp^-1 = X^T X on the matrix cores, one workgroup per (body,
//                64 x 64 tile)
//   (bodies with more than 480 rows: pc_chol / pc_inverse, the unblocked
//   right-looking versions, with X = L^-1 kept transposed in the upper triangle)
//   pc_body      Z_p = M_pp^-1 K_p (m x 6), R_p = K_p^T Z_p, N~_p = R_p^+
//                (cyclic Jacobi eigen-decomposition, eigenvalues below
//                1e-12 * max dropped: the minimum-norm velocity of bodies with
//                a resistance-free motion)
// per assembly a (bodies joined by constraints):
//   pc_asm       S_a = C_a N~_a C_a^T, G~_a = S_a^-1 (by the sweep up to 256 rows,
//                else by Cholesky), or S_a^+ when a pivot falls below 1e-12 * max
//                diagonal (C_a without full row rank)
// Apply (every GMRES iteration), for residual r = (r_lam, r_U, r_phi):
//   pc_apply1    t_p = M_pp^-1 r_lam,p;  U^_p = -N~_p (r_U,p + Z_p^T r_lam,p)
//   pc_apply2    phi_a = G~_a (r_phi,a - C_a U^_a)
//   pc_apply3    U_p = U^_p + N~_p (C^T phi)_p;  lam_p = t_p + Z_p U_p
// which is the exact solution of the body-diagonal saddle problem: row 1 gives
// lam = M~^-1 (r_lam + K U), row 2 gives N~^-1 U = -r_U - K^T M~^-1 r_lam + C^T phi,
// row 3 gives (C N~ C^T) phi = r_phi - C U^.
#include "rpy_device.h"

namespace arb {

constexpr int kMaxBodyBlobs = 512;
constexpr int kMaxM = 3 * kMaxBodyBlobs;
constexpr int kMaxAsmRows = 2048;

// cyclic Jacobi eigen-decomposition of symmetric S (n x n, destroyed) with
// eigenvectors accumulated in V; writes the pseudo-inverse (cutoff relative to
// the largest |eigenvalue|) to out.  Returns the number of dropped eigenvalues.
// Single thread.
__device__ __forceinline__ int sym_pinv_serial(double *S, double *V, int n, double *out,
                                                double cutoff) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < n; ++i) {
            dia += S[i * n + i] * S[i * n + i];
            for (int j = i + 1; j < n; ++j) off += S[i * n + j] * S[i * n + j];
        }
        if (!(off > 1e-32 * dia)) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = S[p * n + q];
                if (apq == 0.0) continue;
                const double tau = (S[q * n + q] - S[p * n + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                for (int k = 0; k < n; ++k) {  // S <- S J
                    const double akp = S[k * n + p], akq = S[k * n + q];
                    S[k * n + p] = c * akp - s * akq;
                    S[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // S <- J^T S
                    const double apk = S[p * n + k], aqk = S[q * n + k];
                    S[p * n + k] = c * apk - s * aqk;
                    S[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V J
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    double wmax = 0.0;
    for (int i = 0; i < n; ++i) wmax = fmax(wmax, fabs(S[i * n + i]));
    const double lim = cutoff * wmax;
    int dropped = 0;
    for (int i = 0; i < n; ++i) {
        const double w = S[i * n + i];
        const double inv = fabs(w) > lim ? 1.0 / w : 0.0;
        dropped += fabs(w) > lim ? 0 : 1;
        S[i * n + i] = inv;  // keep 1/w on the diagonal
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += V[i * n + k] * S[k * n + k] * V[j * n + k];
            out[i * n + j] = s;
        }
    return dropped;
}

__global__ __launch_bounds__(256) void pc_assemble_kernel(const int *__restrict__ blob_off,
                                                          const int64_t *__restrict__ mat_off,
                                                          const double *__restrict__ pos, CoefD c,
                                                          double scale, int wall, double a,
                                                          double *__restrict__ mats,
                                                          int *__restrict__ status) {
    const int p = blockIdx.x;
    const int b0 = blob_off[p], n = blob_off[p + 1] - b0, m = 3 * n;
    double *A = mats + mat_off[p];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx - (idx / n) * n;
        const double *xi = pos + 3 * (size_t)(b0 + i);
        const double *xj = pos + 3 * (size_t)(b0 + j);
        if (wall && i == j && !(xi[2] > a)) atomicOr(&status[2], 1);
        double B[9];
        rpy_block_f64(xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2], xi[2], xj[2], wall != 0, c, B);
        for (int r = 0; r < 3; ++r)
            for (int s = 0; s < 3; ++s) A[(size_t)(3 * i + r) * m + 3 * j + s] = scale * B[3 * r + s];
    }
}

// In-place Cholesky M = L L^T.  Lower triangle: L; upper triangle: L^T (kept
// for coalesced access by pc_inverse); Ldiag receives diag(L).
__global__ __launch_bounds__(256) void pc_chol_kernel(const int *__restrict__ blob_off,
                                                      const int64_t *__restrict__ mat_off,
                                                      double *__restrict__ mats,
                                                      double *__restrict__ ldiag,
                                                      int *__restrict__ status) {
    __shared__ double col[kMaxM];
    __shared__ int fail;
    const int p = blockIdx.x;
    const int m = 3 * (blob_off[p + 1] - blob_off[p]);
    double *A = mats + mat_off[p];
    if (threadIdx.x == 0) fail = 0;
    for (int k = 0; k < m; ++k) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double d = A[(size_t)k * m + k];
            if (!(d > 0.0)) {
                fail = 1;
            } else {
                const double s = sqrt(d);
                A[(size_t)k * m + k] = s;
                col[k] = s;
            }
        }
        __syncthreads();
        if (fail) break;
        const double inv = 1.0 / col[k];
        for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) {
            const double v = A[(size_t)i * m + k] * inv;
            A[(size_t)i * m + k] = v;
            A[(size_t)k * m + i] = v;
            col[i] = v;
        }
        __syncthreads();
        const int w = m - k - 1;
        for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) {
            const int ii = k + 1 + idx / w, jj = k + 1 + (idx - (idx / w) * w);
            A[(size_t)ii * m + jj] -= col[ii] * col[jj];
        }
    }
    __syncthreads();
    if (fail) {
        if (threadIdx.x == 0) atomicMax(&status[0], p + 1);
        return;
    }
    const int b0 = 3 * blob_off[p];
    for (int k = threadIdx.x; k < m; k += blockDim.x) ldiag[b0 + k] = col[k];
}

// X = L^-1 by right-looking forward substitution on the identity, X stored
// as X^T in the upper triangle (the diagonal of X replaces that of L, whose
// diagonal is saved in ldiag); then Minv = X^T X.
__global__ __launch_bounds__(256) void pc_inverse_kernel(const int *__restrict__ blob_off,
                                                         const int64_t *__restrict__ mat_off,
                                                         double *__restrict__ mats,
                                                         const double *__restrict__ ldiag,
                                                         double *__restrict__ minv,
                                                         const int *__restrict__ status) {
    __shared__ double colL[kMaxM];
    __shared__ double rowX[kMaxM];
    const int p = blockIdx.x;
    if (status[0] != 0) return;
    const int m = 3 * (blob_off[p + 1] - blob_off[p]);
    const double *Ld = ldiag + 3 * blob_off[p];
    double *A = mats + mat_off[p];
    double *Mi = minv + mat_off[p];
    // upper triangle incl. diagonal <- identity (X^T)
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int j = idx / m, i = idx - (idx / m) * m;  // element (j, i) = X[i][j]
        if (i >= j) A[(size_t)j * m + i] = (i == j) ? 1.0 : 0.0;
    }
    for (int k = 0; k < m; ++k) {
        __syncthreads();
        const double inv = 1.0 / Ld[k];
        // row k of X: X[k][j], j <= k, lives at A[j*m + k]
        for (int j = threadIdx.x; j <= k; j += blockDim.x) {
            const double v = A[(size_t)j * m + k] * inv;
            A[(size_t)j * m + k] = v;
            rowX[j] = v;
        }
        for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) colL[i] = A[(size_t)i * m + k];
        __syncthreads();
        const int w = m - k - 1;
        const int tot = w * (k + 1);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int j = idx / w, i = k + 1 + (idx - (idx / w) * w);
            A[(size_t)j * m + i] -= colL[i] * rowX[j];
        }
    }
    __syncthreads();
    // Minv[i][j] = sum_{k >= max(i,j)} X[k][i] X[k][j] = sum_k A[i*m+k] A[j*m+k]
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int i = idx / m, j = idx - (idx / m) * m;
        if (j < i) continue;
        const double *ri = A + (size_t)i * m;
        const double *rj = A + (size_t)j * m;
        double s = 0.0;
        for (int k = j; k < m; ++k) s += ri[k] * rj[k];
        Mi[(size_t)i * m + j] = s;
        Mi[(size_t)j * m + i] = s;
    }
}

constexpr int kNB = 32;          // block size of the blocked factorisation
constexpr int kLd = kNB + 1;     // padded LDS row stride (doubles)
constexpr int kFastMaxM = 480;   // largest body handled by the blocked kernels

// FP64 matrix core, one wavefront: D (16 x 16) += A (16 x 4) B (4 x 16).  Lane l
// supplies a = A[l % 16][l / 16] and b = B[l / 16][l % 16] and holds
// D[4 e + l / 16][l % 16] in element e of the accumulator.
typedef double mfma_acc __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mfma_acc mfma_f64_16x16x4(double a, double b, mfma_acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A batch of symmetric positive definite matrices for the blocked kernels:
// matrix p has m_p = scale * (off[p+1] - off[p]) rows (scale 3 for the blob
// mobilities, off = blob offsets; scale 1 for the assemblies' S_a, off = row
// offsets), row-major at mats + mat_off[p]; its diagonal-block inverses at
// dinv_offset.  A matrix whose pivot falls to rel_tol * (its largest diagonal
// entry) or below fails: with fail != nullptr it is flagged there (and skipped
// by the later kernels), else status[0] receives p + 1 (an error).
struct MatBatch {
    const int *off;
    int scale;
    const int64_t *mat_off;
    double *mats;
    double *ldiag;  // diag(L) per row (may be null)
    double *dinv;
    double *out;    // the inverses (same offsets as mats)
    int *status;
    int *fail;
    double rel_tol;
};
__device__ __forceinline__ int mat_rows(const MatBatch &B, int p) {
    return B.scale * (B.off[p + 1] - B.off[p]);
}
__device__ __forceinline__ bool mat_skip(const MatBatch &B, int p) {
    return B.status[0] != 0 || (B.fail && B.fail[p]);
}
// offset (doubles) of matrix p's diagonal-block inverses: 1024 per 32-row block
__device__ __forceinline__ int64_t dinv_offset(const MatBatch &B, int p) {
    return 32 * B.scale * (int64_t)B.off[p] + 1024 * (int64_t)p;
}


// Blocked right-looking Cholesky of each matrix of the batch, in place (lower
// triangle; the upper triangle is not touched), one workgroup per matrix,
// 32-column panels.  Per panel:
//   1. the 32 x 32 diagonal block is factored in LDS (outer-product form: one
//      barrier per pivot, the columns scaled once at the end), and its inverse
//      L_kk^-1 formed by the same row operations on the identity (kept in LDS and
//      stored for the triangular-inverse kernel);
//   2. the rows below become L_bel = A_bel L_kk^-T on the matrix cores (wavefront
//      w takes the 16-row tiles w, w + 4, ...; both column tiles of a row tile in
//      one wavefront, so a row is read completely before it is overwritten), stored
//      in the matrix and, column-major, in a panel scratch: the first 32 m doubles
//      of the matrix's slot in B.out, which only the later kernels write;
//   3. the trailing lower triangle takes A -= L_bel L_bel^T on the matrix cores in
//      64 x 64 tiles (wavefront w: the 32 x 32 quarter (w / 2, w % 2)), operands
//      read from the scratch (16 consecutive rows per load); a tile's entries are
//      read before its products run.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void pc_potrf_kernel(
    MatBatch B) {
    __shared__ double Dk[kNB * kLd];  // diagonal block, then L_kk
    __shared__ double Wi[kNB * kLd];  // L_kk^-1, zero padded
    __shared__ double isq[kNB];
    __shared__ int fail;
    __shared__ double piv_tol;
    const int p = blockIdx.x, tid = threadIdx.x;
    if (mat_skip(B, p)) return;
    const int m = mat_rows(B, p);
    double *A = B.mats + B.mat_off[p];
    double *Lp = B.out + B.mat_off[p];  // panel scratch, Lp[t * m + i]
    double *Dg = B.dinv + dinv_offset(B, p);
    const int w = tid >> 6, l = tid & 63;
    if (tid == 0) {
        fail = 0;
        double dmax = 0.0;
        if (B.rel_tol > 0.0)
            for (int k = 0; k < m; ++k) dmax = fmax(dmax, A[(size_t)k * m + k]);
        piv_tol = B.rel_tol * dmax;
    }
    for (int k0 = 0; k0 < m; k0 += kNB) {
        const int nb = min(kNB, m - k0), nt = m - k0 - nb;  // nt rows below the block
        __syncthreads();
        // 1. the diagonal block: thread tid holds entries (i, c) = (tid / 32 + 8 q, tid % 32).
        // The row operations of the elimination (row i -= l_ij row j, l_ij = D_ij / D_jj)
        // are applied to the identity in Wi as well, which turns it into the unit lower
        // triangular inverse factor; scaled by the pivots' 1/sqrt it is L_kk^-1
        const int c = tid & 31;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = (tid >> 5) + 8 * q;
            Dk[i * kLd + c] = (i < nb && c <= i) ? A[(size_t)(k0 + i) * m + k0 + c] : 0.0;
            Wi[i * kLd + c] = (i < nb && c == i) ? 1.0 : 0.0;
        }
        __syncthreads();
        bool bad = false;
        for (int j = 0; j < nb; ++j) {
            const double d = Dk[j * kLd + j];
            if (!(d > piv_tol)) {  // the same value for every thread: a uniform exit
                bad = true;
                break;
            }
            const double inv = 1.0 / d;
            // the pivot-row factor of this thread's column, then its four entries
            // (loads in bounds and unconditional; stores only below the pivot)
            const bool right = c > j;
            double *X = right ? Dk : Wi;
            const double pj = (right ? Dk[c * kLd + j] : Wi[j * kLd + c]) * inv;
            double lij[4], xv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = (tid >> 5) + 8 * q;
                lij[q] = Dk[i * kLd + j];
                xv[q] = X[i * kLd + c];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = (tid >> 5) + 8 * q;
                if (i > j && i < nb && (!right || c <= i)) X[i * kLd + c] = xv[q] - lij[q] * pj;
            }
            __syncthreads();
        }
        if (bad) {
            if (tid == 0) fail = 1;
            break;
        }
        // L_ic = D_ic / sqrt(D_cc), (L^-1)_ic = E_ic / sqrt(D_ii) with the final pivots D
        if (tid < nb) isq[tid] = 1.0 / sqrt(Dk[tid * kLd + tid]);
        __syncthreads();
        double lv[4], xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = (tid >> 5) + 8 * q;
            const bool in = i < nb && c <= i;
            lv[q] = in ? Dk[i * kLd + c] * isq[c] : 0.0;
            xv[q] = in ? Wi[i * kLd + c] * isq[i] : 0.0;
        }
        __syncthreads();
        double *Db = Dg + (k0 / kNB) * (kNB * kNB);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = (tid >> 5) + 8 * q;
            Dk[i * kLd + c] = lv[q];
            Wi[i * kLd + c] = xv[q];
            Db[i * kNB + c] = xv[q];
            if (i < nb && c <= i) A[(size_t)(k0 + i) * m + k0 + c] = lv[q];
            if (B.ldiag && i < nb && c == i) B.ldiag[B.scale * (int64_t)B.off[p] + k0 + i] = lv[q];
        }
        if (nt <= 0) break;  // the last panel (nb = 32 whenever rows remain below)
        __syncthreads();
        // 2. L_bel = A_bel L_kk^-T: tile (row tile rt, column tile ct), lane l supplies
        // a = A_bel[16 rt + l % 16][4 s + l / 16] and b = Wi[16 ct + l % 16][4 s + l / 16]
        const int nrt = (nt + 15) >> 4;
        double *Abel = A + (size_t)(k0 + kNB) * m + k0;
        for (int rt = w; rt < nrt; rt += 4) {
            const int ra = min(16 * rt + (l & 15), nt - 1);
            double av[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) av[s] = Abel[(size_t)ra * m + 4 * s + (l >> 4)];
            mfma_acc acc0 = {}, acc1 = {};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int kk = 4 * s + (l >> 4);
                acc0 = mfma_f64_16x16x4(av[s], Wi[(l & 15) * kLd + kk], acc0);
                acc1 = mfma_f64_16x16x4(av[s], Wi[(16 + (l & 15)) * kLd + kk], acc1);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * rt + 4 * e + (l >> 4);
                if (i < nt) {
                    const int cc = l & 15;
                    Abel[(size_t)i * m + cc] = acc0[e];
                    Abel[(size_t)i * m + 16 + cc] = acc1[e];
                    Lp[(size_t)cc * m + i] = acc0[e];
                    Lp[(size_t)(16 + cc) * m + i] = acc1[e];
                }
            }
        }
        __syncthreads();
        // 3. trailing update of the lower triangle, A_ij -= sum_t L_it L_jt
        const int t0 = k0 + kNB;
        const int ntile = (nt + 63) / 64;
        const int wr = w >> 1, wc = w & 1;
        const int ntiles = ntile * (ntile + 1) / 2;
        // tile -> (bi, bj), bj <= bi, row by row of the lower triangle of tiles
        auto tile_ij = [](int tile, int &bi, int &bj) {
            bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
            bj = tile - bi * (bi + 1) / 2;
        };
        // this lane's 16 entries of a tile's 32 x 32 quarter (clamped into the matrix)
        auto load_quarter = [&](int i0, int j0, double (&v)[2][2][4]) {
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int i = min(i0 + 16 * ti + 4 * e + (l >> 4), nt - 1);
                        const int j = min(j0 + 16 * tj + (l & 15), nt - 1);
                        v[ti][tj][e] = A[(size_t)(t0 + i) * m + t0 + j];
                    }
        };
        for (int tile = 0; tile < ntiles; ++tile) {
            int bi, bj;
            tile_ij(tile, bi, bj);
            const int i0 = 64 * bi + 32 * wr, j0 = 64 * bj + 32 * wc;
            double cur[2][2][4];
            load_quarter(i0, j0, cur);
            const int ra0 = min(i0 + (l & 15), nt - 1), ra1 = min(i0 + 16 + (l & 15), nt - 1);
            const int rb0 = min(j0 + (l & 15), nt - 1), rb1 = min(j0 + 16 + (l & 15), nt - 1);
            mfma_acc acc[2][2] = {};
#pragma unroll 2
            for (int s = 0; s < 8; ++s) {
                const double *col = Lp + (size_t)(4 * s + (l >> 4)) * m;
                const double a0 = col[ra0], a1 = col[ra1], b0 = col[rb0], b1 = col[rb1];
                acc[0][0] = mfma_f64_16x16x4(a0, b0, acc[0][0]);
                acc[0][1] = mfma_f64_16x16x4(a0, b1, acc[0][1]);
                acc[1][0] = mfma_f64_16x16x4(a1, b0, acc[1][0]);
                acc[1][1] = mfma_f64_16x16x4(a1, b1, acc[1][1]);
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int i = i0 + 16 * ti + 4 * e + (l >> 4);
                        const int j = j0 + 16 * tj + (l & 15);
                        if (i < nt && j <= i)
                            A[(size_t)(t0 + i) * m + t0 + j] = cur[ti][tj][e] - acc[ti][tj][e];
                    }
        }
    }
    __syncthreads();
    if (fail && tid == 0) {
        if (B.fail)
            B.fail[p] = 1;
        else
            atomicMax(&B.status[0], p + 1);
    }
}

// load (4 per thread) the 32 x 32 block of L at (R0, C0), zero padded beyond m
__device__ __forceinline__ void load_block(double v[4], const double *A, int m, int R0, int C0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 256 * e, t = idx / kNB, u = idx % kNB;
        v[e] = (R0 + t < m && C0 + u < m) ? A[(size_t)(R0 + t) * m + C0 + u] : 0.0;
    }
}
__device__ __forceinline__ void store_block(double (*Ls)[kLd], const double v[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 256 * e;
        Ls[idx / kNB][idx % kNB] = v[e];
    }
}

// X = L^-1, block column [32 cb, 32 cb + 32): forward block substitution on the
// identity, X_i = Dinv_i (E_i - sum_{cb <= k < i} L_ik X_k); the next block of
// L is read into registers while the current one is used.  The strictly lower
// part of X is stored transposed in the strictly upper triangle of M_pp's
// storage (the diagonal of X is 1 / diag(L)).  Dynamic LDS: the block column,
// ceil(max_m / 32) * 32 x kLd doubles.
__global__ __launch_bounds__(256) void pc_trtri_kernel(MatBatch B) {
    extern __shared__ double X[];
    __shared__ double Ls[kNB][kLd];
    const int p = blockIdx.y, cb = blockIdx.x;
    if (mat_skip(B, p)) return;
    const int m = mat_rows(B, p);
    const int nbk = (m + kNB - 1) / kNB;
    if (cb >= nbk) return;
    double *A = B.mats + B.mat_off[p];
    const double *Dg = B.dinv + dinv_offset(B, p);
    // wavefront w holds the 16 x 16 tile (w / 2, w % 2) of each 32 x 32 block step
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int wr = 16 * (w >> 1), wc = 16 * (w & 1);
    const int lr = l & 15, lk = l >> 4;  // operand row and k offset of this lane
    const int c0 = kNB * cb;
    for (int i = cb; i < nbk; ++i) {
        double dreg[4], nxt[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) dreg[e] = Dg[(size_t)i * kNB * kNB + tid + 256 * e];
        if (cb < i) load_block(nxt, A, m, kNB * i, kNB * cb);
        mfma_acc acc;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = (kNB * i + wr + 4 * e + lk == c0 + wc + lr) ? 1.0 : 0.0;
        for (int k = cb; k < i; ++k) {
            __syncthreads();
            store_block(Ls, nxt);
            __syncthreads();
            if (k + 1 < i) load_block(nxt, A, m, kNB * i, kNB * (k + 1));
            const double *Xk = X + (size_t)kNB * k * kLd + wc + lr;
#pragma unroll
            for (int kk = 0; kk < kNB; kk += 4)
                acc = mfma_f64_16x16x4(-Ls[wr + lr][kk + lk], Xk[(kk + lk) * kLd], acc);
        }
        double *Xi = X + (size_t)kNB * i * kLd;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) Xi[(wr + 4 * e + lk) * kLd + wc + lr] = acc[e];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + 256 * e;
            Ls[idx / kNB][idx % kNB] = dreg[e];
        }
        __syncthreads();
        mfma_acc y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < kNB; kk += 4)
            y = mfma_f64_16x16x4(Ls[wr + lr][kk + lk], Xi[(kk + lk) * kLd + wc + lr], y);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) Xi[(wr + 4 * e + lk) * kLd + wc + lr] = y[e];
    }
    __syncthreads();
    // X[i][c0 + c] for i > c0 + c  ->  A[(c0 + c) m + i]  (consecutive i: coalesced)
    const int rows = m - c0;
    for (int idx = tid; idx < rows * kNB; idx += 256) {
        const int c = idx / rows, i = c0 + idx % rows;
        const int j = c0 + c;
        if (j < m && i > j) A[(size_t)j * m + i] = X[(size_t)i * kLd + c];
    }
}

// M_pp^-1 = X^T X = U U^T with U = X^T upper triangular (strictly upper part in
// M_pp's storage; the diagonal, 1 / diag(L), read from the diagonal-block
// inverses).  One workgroup per (body, 64 x 64 tile (I, J), I <= J); the sum
// over k >= J runs in chunks of 32 staged in LDS, the next chunk read into
// registers meanwhile.  Writes both (I, J) and (J, I).
__global__ __launch_bounds__(256) void pc_lauum_kernel(MatBatch B) {
    __shared__ double Ua[64][kLd], Ub[64][kLd];
    const int p = blockIdx.y;
    if (mat_skip(B, p)) return;
    const int m = mat_rows(B, p);
    const int nt = (m + 63) / 64;
    const int tile = blockIdx.x;
    if (tile >= nt * (nt + 1) / 2) return;
    int bj = 0;
    while ((bj + 1) * (bj + 2) / 2 <= tile) ++bj;
    const int bi = tile - bj * (bj + 1) / 2;  // bi <= bj
    const int I0 = 64 * bi, J0 = 64 * bj;
    const double *A = B.mats + B.mat_off[p];
    const double *Dg = B.dinv + dinv_offset(B, p);
    double *Mi = B.out + B.mat_off[p];
    const int tid = threadIdx.x;
    const int kl = tid & 31, r0 = tid >> 5;  // a thread stages column kl of rows r0 + 8e
    // wavefront w computes the 32 x 32 quarter (w / 2, w % 2) as 2 x 2 matrix-core tiles
    const int w = tid >> 6, l = tid & 63, wr = 32 * (w >> 1), wc = 32 * (w & 1);
    const int lr = l & 15, lk = l >> 4;
    // U[row][kk]: 0 below the diagonal, 1/L_kk on it, X[kk][row] above
    auto u_at = [&](int row, int kk) -> double {
        if (row >= m || kk >= m || kk < row) return 0.0;
        if (kk == row) return Dg[(size_t)(row >> 5) * kNB * kNB + (row & 31) * (kNB + 1)];
        return A[(size_t)row * m + kk];
    };
    double na[8], nb8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        na[e] = u_at(I0 + r0 + 8 * e, J0 + kl);
        nb8[e] = u_at(J0 + r0 + 8 * e, J0 + kl);
    }
    mfma_acc acc[2][2] = {};
    for (int k0 = J0; k0 < m; k0 += kNB) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            Ua[r0 + 8 * e][kl] = na[e];
            Ub[r0 + 8 * e][kl] = nb8[e];
        }
        __syncthreads();
        if (k0 + kNB < m) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                na[e] = u_at(I0 + r0 + 8 * e, k0 + kNB + kl);
                nb8[e] = u_at(J0 + r0 + 8 * e, k0 + kNB + kl);
            }
        }
#pragma unroll
        for (int kk = 0; kk < kNB; kk += 4) {
            const double a0 = Ua[wr + lr][kk + lk], a1 = Ua[wr + 16 + lr][kk + lk];
            const double b0 = Ub[wc + lr][kk + lk], b1 = Ub[wc + 16 + lr][kk + lk];
            acc[0][0] = mfma_f64_16x16x4(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f64_16x16x4(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f64_16x16x4(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f64_16x16x4(a1, b1, acc[1][1]);
        }
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = I0 + wr + 16 * ti + 4 * e + lk;
                const int j = J0 + wc + 16 * tj + lr;
                if (i < m && j < m) {
                    Mi[(size_t)i * m + j] = acc[ti][tj][e];
                    Mi[(size_t)j * m + i] = acc[ti][tj][e];
                }
            }
}

// restore L's diagonal (for inspection) once the inverse no longer needs X
__global__ void pc_restore_diag_kernel(const int *__restrict__ blob_off,
                                       const int64_t *__restrict__ mat_off,
                                       double *__restrict__ mats,
                                       const double *__restrict__ ldiag) {
    const int p = blockIdx.x;
    const int m = 3 * (blob_off[p + 1] - blob_off[p]);
    double *A = mats + mat_off[p];
    for (int k = threadIdx.x; k < m; k += blockDim.x)
        A[(size_t)k * m + k] = ldiag[3 * blob_off[p] + k];
}

// rows of K_p: blob i, component a: u part e_a, w part row a of -(d_i^x)
__device__ __forceinline__ double K_entry(const double *d, int a, int c) {
    if (c < 3) return a == c ? 1.0 : 0.0;
    const int b = c - 3;
    // -(d^x)[a][b] with d^x = [[0,-d2,d1],[d2,0,-d0],[-d1,d0,0]]
    if (a == b) return 0.0;
    if (a == 0) return b == 1 ? d[2] : -d[1];
    if (a == 1) return b == 0 ? -d[2] : d[0];
    return b == 0 ? d[1] : -d[0];
}

// out = R^-1 for a symmetric positive definite 6 x 6 R by Cholesky (R = L L^T,
// X = L^-1, R^-1 = X^T X; L and X are 36-double scratch, row-major); false,
// with out untouched, when a pivot falls to 1e-8 of the largest diagonal entry
// or below (then the caller takes the pseudo-inverse, which is the inverse
// whenever this succeeds)
__device__ inline bool chol_inv6(const double *R, double *L, double *X, double *out) {
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i) dmax = fmax(dmax, R[i * 6 + i]);
    const double tol = 1e-8 * dmax;
    for (int j = 0; j < 6; ++j) {
        double d = R[j * 6 + j];
        for (int k = 0; k < j; ++k) d -= L[j * 6 + k] * L[j * 6 + k];
        if (!(d > tol)) return false;
        L[j * 6 + j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = R[i * 6 + j];
            for (int k = 0; k < j; ++k) v -= L[i * 6 + k] * L[j * 6 + k];
            L[i * 6 + j] = v / L[j * 6 + j];
        }
    }
    for (int c = 0; c < 6; ++c)
        for (int i = 0; i < 6; ++i) {
            if (i < c) {
                X[i * 6 + c] = 0.0;
                continue;
            }
            double v = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= L[i * 6 + k] * X[k * 6 + c];
            X[i * 6 + c] = v / L[i * 6 + i];
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double v = 0.0;
            for (int k = max(i, j); k < 6; ++k) v += X[k * 6 + i] * X[k * 6 + j];
            out[i * 6 + j] = v;
        }
    return true;
}

// Per body: Z = M^-1 K (m x 6) and N~ = (K^T M^-1 K)^-1 (Sec. 3.1).  Thread r
// takes row r of Z (M^-1 is symmetric, so the row is read as column r:
// consecutive threads read consecutive addresses) and adds K_r^T Z_r to its
// partial R = K^T Z (the 21 entries of the upper triangle); the partials are
// summed over the wavefronts, then N~ = R^-1 by Cholesky; when R is singular (a
// rod of collinear blobs) R is stored and flagged for pc_body_pinv_kernel.
__global__ __launch_bounds__(256) void pc_body_kernel(const int *__restrict__ blob_off,
                                                      const int64_t *__restrict__ mat_off,
                                                      const int64_t *__restrict__ z_off,
                                                      const double *__restrict__ minv,
                                                      const double *__restrict__ dvec,
                                                      double *__restrict__ Zbuf,
                                                      double *__restrict__ Nt,
                                                      int *__restrict__ body_pinv,
                                                      int *__restrict__ status) {
    __shared__ double red[4][21];
    __shared__ double S6[36], V6[36], L6[36];  // R, then Cholesky scratch
    const int p = blockIdx.x;
    if (status[0] != 0) return;
    const int b0 = blob_off[p], n = blob_off[p + 1] - b0, m = 3 * n;
    const double *Mi = minv + mat_off[p];
    double *Z = Zbuf + z_off[p];
    const double *d = dvec + 3 * (size_t)b0;
    double racc[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) racc[e] = 0.0;
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        double z[6] = {0, 0, 0, 0, 0, 0};
        const double *col = Mi + r;
        for (int i = 0; i < n; ++i) {
            const double m0 = col[(size_t)(3 * i) * m], m1 = col[(size_t)(3 * i + 1) * m],
                         m2 = col[(size_t)(3 * i + 2) * m];
            const double *di = d + 3 * i;
            z[0] += m0;
            z[1] += m1;
            z[2] += m2;
            // sum_a M[r][3i+a] * (-(d^x))[a][b]
            z[3] += -m1 * di[2] + m2 * di[1];
            z[4] += m0 * di[2] - m2 * di[0];
            z[5] += -m0 * di[1] + m1 * di[0];
        }
        for (int c = 0; c < 6; ++c) Z[(size_t)r * 6 + c] = z[c];
        // row r = 3 i + a of K: e_a, then -(d_i^x) row a
        const double *dr = d + 3 * (r / 3);
        const int a = r % 3;
        double kr[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) kr[c] = K_entry(dr, a, c);
        int e = 0;
#pragma unroll
        for (int c1 = 0; c1 < 6; ++c1)
#pragma unroll
            for (int c2 = c1; c2 < 6; ++c2) racc[e++] += kr[c1] * z[c2];
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < 21; ++e) {
        double v = racc[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[w][e] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int e = 0;
        for (int c1 = 0; c1 < 6; ++c1)
            for (int c2 = c1; c2 < 6; ++c2, ++e) {
                double v = 0.0;
                for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += red[k][e];
                S6[c1 * 6 + c2] = v;
                S6[c2 * 6 + c1] = v;
            }
        double *out = Nt + 36 * (size_t)p;
        const bool ok = chol_inv6(S6, L6, V6, out);
        if (!ok)  // R for pc_body_pinv_kernel
            for (int k = 0; k < 36; ++k) out[k] = S6[k];
        body_pinv[p] = ok ? 0 : 1;
    }
}

// N~_p = R_p^+ (symmetric pseudo-inverse, eigenvalues below 1e-12 of the largest
// dropped) for the bodies whose R_p failed the Cholesky test, one thread each
__global__ __launch_bounds__(64) void pc_body_pinv_kernel(int M, const int *__restrict__ body_pinv,
                                                          double *__restrict__ Nt,
                                                          int *__restrict__ status) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M || !body_pinv[p] || status[0] != 0) return;
    double S[36], V[36];
    double *out = Nt + 36 * (size_t)p;
    for (int k = 0; k < 36; ++k) S[k] = out[k];
    if (sym_pinv_serial(S, V, 6, out, 1e-12)) atomicAdd(&status[3], 1);
}

// S = C_a N~_a C_a^T (na x na, row-major) for the assembly's rows r0 .. r0+na-1,
// all threads of the block
__device__ void asm_form_S(int r0, int na, const int *__restrict__ asm_rows,
                           const int *__restrict__ row_p, const int *__restrict__ row_q,
                           const double *__restrict__ crow, const double *__restrict__ Nt,
                           double *__restrict__ S) {
    for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
        const int k = idx / na, l = idx - (idx / na) * na;
        const int rk = asm_rows[r0 + k], rl = asm_rows[r0 + l];
        double sum = 0.0;
#pragma unroll 1
        for (int sk = 0; sk < 2; ++sk) {
            const int bk = sk ? row_q[rk] : row_p[rk];
            if (bk < 0) continue;
            const double *ck = crow + 12 * (size_t)rk + 6 * sk;
#pragma unroll 1
            for (int sl = 0; sl < 2; ++sl) {
                const int bl = sl ? row_q[rl] : row_p[rl];
                if (bl != bk) continue;
                const double *cl = crow + 12 * (size_t)rl + 6 * sl;
                const double *Nb = Nt + 36 * (size_t)bk;
                for (int u = 0; u < 6; ++u) {
                    double t = 0.0;
                    for (int v = 0; v < 6; ++v) t += Nb[u * 6 + v] * cl[v];
                    sum += ck[u] * t;
                }
            }
        }
        S[(size_t)k * na + l] = sum;
    }
}

// The rows of one assembly staged in LDS: cl[12 k + 6 side + u] the row's
// coefficients on the body of that side, bl[2 k + side] the body (-1: none).
__device__ void asm_stage_rows(int r0, int na, const int *__restrict__ asm_rows,
                               const int *__restrict__ row_p, const int *__restrict__ row_q,
                               const double *__restrict__ crow, double *cl, int *bl) {
    for (int idx = threadIdx.x; idx < 12 * na; idx += blockDim.x) {
        const int k = idx / 12, u = idx - 12 * k;
        cl[idx] = crow[12 * (size_t)asm_rows[r0 + k] + u];
    }
    for (int k = threadIdx.x; k < na; k += blockDim.x) {
        const int rk = asm_rows[r0 + k];
        bl[2 * k] = row_p[rk];
        bl[2 * k + 1] = row_q[rk];
    }
}

// Column l of the lower triangle of S_a = C_a N~ C_a^T from the staged rows, by
// the calling thread: t_side = N~_b c_l,side for the bodies b of row l, then
// S_kl = sum of c_k,side' . t_side over the side pairs on the same body, k >= l.
// store(k, value) receives every entry.  The rows are visited from k = 0 (the
// threads of a wavefront store row k together, at consecutive addresses); rows
// above the diagonal are skipped.
template <class F>
__device__ __forceinline__ void asm_column(int l, int na, const double *cl, const int *bl,
                                           const double *__restrict__ Nt, F &&store) {
    double t[2][6];
    int bs[2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        bs[sd] = bl[2 * l + sd];
        const double *c = cl + 12 * l + 6 * sd;
        const double *Nb = Nt + 36 * (size_t)max(bs[sd], 0);
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            double v = 0.0;
            if (bs[sd] >= 0)
#pragma unroll
                for (int w = 0; w < 6; ++w) v += Nb[u * 6 + w] * c[w];
            t[sd][u] = v;
        }
    }
    for (int k = 0; k < na; ++k) {
        if (k < l) continue;
        const int b0 = bl[2 * k], b1 = bl[2 * k + 1];
        double sum = 0.0;
#pragma unroll
        for (int sk = 0; sk < 2; ++sk) {
            const int bk = sk ? b1 : b0;
            if (bk < 0) continue;
            const double *c = cl + 12 * k + 6 * sk;
#pragma unroll
            for (int sd = 0; sd < 2; ++sd)
                if (bk == bs[sd])
#pragma unroll
                    for (int u = 0; u < 6; ++u) sum += c[u] * t[sd][u];
        }
        store(k, sum);
    }
}

// the lower triangle of the assemblies' S_a for the blocked kernels (assemblies of
// at most kFastMaxM rows; the factorisation reads no other entries).  Dynamic LDS:
// the staged rows, 12 doubles and 2 ints per row of the largest assembly.
__global__ __launch_bounds__(256) void pc_asm_form_kernel(
    const int *__restrict__ asm_row_ptr, const int *__restrict__ asm_rows,
    const int64_t *__restrict__ asm_mat_off, const int *__restrict__ row_p,
    const int *__restrict__ row_q, const double *__restrict__ crow, const double *__restrict__ Nt,
    double *__restrict__ Sbuf, int *__restrict__ fail, const int *__restrict__ status,
    int max_rows) {
    extern __shared__ double sm[];
    double *cl = sm;
    int *bl = reinterpret_cast<int *>(sm + 12 * (size_t)max_rows);
    const int a = blockIdx.x;
    const int r0 = asm_row_ptr[a], na = asm_row_ptr[a + 1] - r0;
    if (threadIdx.x == 0) fail[a] = 0;
    if (na == 0 || status[0] != 0) return;
    asm_stage_rows(r0, na, asm_rows, row_p, row_q, crow, cl, bl);
    __syncthreads();
    double *S = Sbuf + asm_mat_off[a];
    for (int l = threadIdx.x; l < na; l += blockDim.x)
        asm_column(l, na, cl, bl, Nt, [&](int k, double v) { S[(size_t)k * na + l] = v; });
}

// assemblies whose S_a failed the Cholesky pivot test: S_a formed again and its
// symmetric pseudo-inverse (eigenvalues below 1e-12 * max dropped), Sec. 3.1;
// X is scratch of na^2 doubles after S in the same assembly slot of Xbuf
__global__ __launch_bounds__(256) void pc_asm_pinv_kernel(
    const int *__restrict__ asm_row_ptr, const int *__restrict__ asm_rows,
    const int64_t *__restrict__ asm_mat_off, const int *__restrict__ row_p,
    const int *__restrict__ row_q, const double *__restrict__ crow, const double *__restrict__ Nt,
    double *__restrict__ Xbuf, double *__restrict__ Gbuf, const int *__restrict__ fail,
    int *__restrict__ status) {
    const int a = blockIdx.x;
    if (!fail[a] || status[0] != 0) return;
    const int r0 = asm_row_ptr[a], na = asm_row_ptr[a + 1] - r0;
    double *S = Xbuf + 2 * asm_mat_off[a];
    asm_form_S(r0, na, asm_rows, row_p, row_q, crow, Nt, S);
    __syncthreads();
    if (threadIdx.x == 0) {
        sym_pinv_serial(S, S + (size_t)na * na, na, Gbuf + asm_mat_off[a], 1e-12);
        atomicAdd(&status[1], 1);
    }
}

// Assemblies of at most kAsmSmall rows, one workgroup of 1,024 threads each,
// everything in LDS (dynamic: S and E, n (n + 1) doubles each, the staged rows and
// N~_b c per row, for n rows of the largest assembly):
//   S = C_a N~ C_a^T (lower triangle, an entry per thread);
//   elimination in outer-product form (row i -= l_ij row j, l_ij = S_ij / S_jj,
//   one barrier per pivot; pivot test relative to the largest diagonal entry),
//   the same row operations applied to the identity in E, which becomes the unit
//   lower triangular factor E with E S E^T = D (the final pivots);
//   G~ = S^-1 = E^T D^-1 E, each entry by one thread.
// A failed pivot flags the assembly for the pseudo-inverse kernel.
constexpr int kAsmSmall = 64;
constexpr int kAsmThreads = 1024;
constexpr int kAsmSlots = kAsmSmall * kAsmSmall / kAsmThreads;  // rows per thread
__global__ __launch_bounds__(kAsmThreads) void pc_asm_small_kernel(
    const int *__restrict__ asm_row_ptr, const int *__restrict__ asm_rows,
    const int64_t *__restrict__ asm_mat_off, const int *__restrict__ row_p,
    const int *__restrict__ row_q, const double *__restrict__ crow, const double *__restrict__ Nt,
    double *__restrict__ Gbuf, int *__restrict__ fail, const int *__restrict__ status,
    int max_rows) {
    extern __shared__ double sm[];
    const int ld = max_rows + 1;
    double *S = sm, *E = S + (size_t)max_rows * ld, *cl = E + (size_t)max_rows * ld;
    double *tl = cl + 12 * (size_t)max_rows;  // N~_b c for both sides of each row
    int *bl = reinterpret_cast<int *>(tl + 12 * (size_t)max_rows);
    __shared__ double tol;
    __shared__ double invd[kAsmSmall];
    const int a = blockIdx.x, tid = threadIdx.x;
    const int r0 = asm_row_ptr[a], na = asm_row_ptr[a + 1] - r0;
    if (tid == 0) fail[a] = 0;
    if (na == 0 || status[0] != 0) return;
    asm_stage_rows(r0, na, asm_rows, row_p, row_q, crow, cl, bl);
    for (int idx = tid; idx < kAsmSmall * kAsmSmall; idx += kAsmThreads) {
        const int i = idx >> 6, c = idx & 63;
        if (i < na && c <= i) E[i * ld + c] = i == c ? 1.0 : 0.0;
    }
    __syncthreads();
    // t = N~_b c per row and side (a thread per entry), then every entry of the
    // lower triangle of S = C N~ C^T at once
    for (int idx = tid; idx < 12 * na; idx += kAsmThreads) {
        const int l = idx / 12, sd = (idx / 6) & 1, u = idx % 6;
        const int b = bl[2 * l + sd];
        double v = 0.0;
        if (b >= 0)
            for (int w = 0; w < 6; ++w) v += Nt[36 * (size_t)b + u * 6 + w] * cl[12 * l + 6 * sd + w];
        tl[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < kAsmSmall * kAsmSmall; idx += kAsmThreads) {
        const int k = idx >> 6, l = idx & 63;
        if (k >= na || l > k) continue;
        double sum = 0.0;
        for (int sk = 0; sk < 2; ++sk) {
            const int bk = bl[2 * k + sk];
            if (bk < 0) continue;
            for (int sl = 0; sl < 2; ++sl)
                if (bl[2 * l + sl] == bk)
                    for (int u = 0; u < 6; ++u)
                        sum += cl[12 * k + 6 * sk + u] * tl[12 * l + 6 * sl + u];
        }
        S[k * ld + l] = sum;
    }
    __syncthreads();
    if (tid == 0) {
        double dmax = 0.0;
        for (int k = 0; k < na; ++k) dmax = fmax(dmax, S[k * ld + k]);
        tol = 1e-12 * dmax;
    }
    __syncthreads();
    // thread tid owns column c = tid % 64 of rows i = tid / 64 + 16 q (q < kAsmSlots):
    // the column-c entries of row j are read once per pivot, the rows' entries all
    // issued before they are updated
    const int c = tid & 63, i0 = tid >> 6;
    for (int j = 0; j < na; ++j) {
        const double d = S[j * ld + j];
        if (!(d > tol)) {  // the same value for every thread: a uniform exit
            if (tid == 0) fail[a] = 1;
            return;
        }
        const double inv = 1.0 / d;
        if (c < na) {
            const bool right = c > j;  // S entry (right of the pivot column), else E entry
            const double pj = (right ? S[c * ld + j] : E[j * ld + c]) * inv;
            double *X = right ? S : E;
            // every load in bounds (rows clamped to the matrix) and issued before
            // the updates, which only the slots below the pivot row store
            double sij[kAsmSlots], xv[kAsmSlots];
#pragma unroll
            for (int q = 0; q < kAsmSlots; ++q) {
                const int i = min(i0 + 16 * q, na - 1);
                sij[q] = S[i * ld + j];
                xv[q] = X[i * ld + c];
            }
#pragma unroll
            for (int q = 0; q < kAsmSlots; ++q) {
                const int i = i0 + 16 * q;
                if (i > j && i < na && c <= i) X[i * ld + c] = xv[q] - sij[q] * pj;
            }
        }
        __syncthreads();
    }
    if (tid < na) invd[tid] = 1.0 / S[tid * ld + tid];
    __syncthreads();
    // G~_ij = sum_k E_ki E_kj / D_k over k >= max(i, j): thread tid takes column
    // j = tid % 64 of rows i = tid / 64 + 16 q, one pass over k
    double *G = Gbuf + asm_mat_off[a];
    const int j = c;
    double acc[kAsmSlots];
#pragma unroll
    for (int q = 0; q < kAsmSlots; ++q) acc[q] = 0.0;
    if (j < na)
        for (int k = j; k < na; ++k) {
            const double ekj = E[k * ld + j] * invd[k];
#pragma unroll
            for (int q = 0; q < kAsmSlots; ++q) {
                const int i = i0 + 16 * q;
                const double eki = E[k * ld + min(i, k)];  // in bounds; used for i <= k
                acc[q] += i <= k ? eki * ekj : 0.0;
            }
        }
#pragma unroll
    for (int q = 0; q < kAsmSlots; ++q) {
        const int i = i0 + 16 * q;
        if (i < na && j < na) G[(size_t)i * na + j] = acc[q];
    }
}

// assemblies beyond kFastMaxM rows: unblocked Cholesky and inverse in global memory
__global__ __launch_bounds__(256) void pc_asm_kernel(
    const int *__restrict__ asm_row_ptr, const int *__restrict__ asm_rows,
    const int64_t *__restrict__ asm_mat_off, const int *__restrict__ row_p,
    const int *__restrict__ row_q, const double *__restrict__ crow, const double *__restrict__ Nt,
    double *__restrict__ Sbuf, double *__restrict__ Gbuf, int *__restrict__ status) {
    __shared__ double col[kMaxAsmRows];
    __shared__ int fail;
    __shared__ double dmax;
    const int a = blockIdx.x;
    const int r0 = asm_row_ptr[a], na = asm_row_ptr[a + 1] - r0;
    if (na == 0) return;
    if (status[0] != 0) return;
    double *S = Sbuf + 2 * asm_mat_off[a];
    double *X = S + (size_t)na * na;
    double *G = Gbuf + asm_mat_off[a];
    for (int pass = 0; pass < 2; ++pass) {
        // S = C_a N~ C_a^T
        asm_form_S(r0, na, asm_rows, row_p, row_q, crow, Nt, S);
        __syncthreads();
        if (pass == 1) {
            // rank-deficient: symmetric pseudo-inverse (Sec. 3.1)
            if (threadIdx.x == 0) {
                sym_pinv_serial(S, X, na, G, 1e-12);
                atomicAdd(&status[1], 1);
            }
            return;
        }
        if (threadIdx.x == 0) {
            double mx = 0.0;
            for (int k = 0; k < na; ++k) mx = fmax(mx, S[(size_t)k * na + k]);
            dmax = mx;
            fail = 0;
        }
        // Cholesky in place (lower = L, upper = L^T), pivot test relative to max diagonal
        for (int k = 0; k < na; ++k) {
            __syncthreads();
            if (threadIdx.x == 0) {
                const double dd = S[(size_t)k * na + k];
                if (!(dd > 1e-12 * dmax)) {
                    fail = 1;
                } else {
                    const double s = sqrt(dd);
                    S[(size_t)k * na + k] = s;
                    col[k] = s;
                }
            }
            __syncthreads();
            if (fail) break;
            const double inv = 1.0 / col[k];
            for (int i = k + 1 + threadIdx.x; i < na; i += blockDim.x) {
                const double v = S[(size_t)i * na + k] * inv;
                S[(size_t)i * na + k] = v;
                S[(size_t)k * na + i] = v;
                col[i] = v;
            }
            __syncthreads();
            const int w = na - k - 1;
            for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) {
                const int ii = k + 1 + idx / w, jj = k + 1 + (idx - (idx / w) * w);
                S[(size_t)ii * na + jj] -= col[ii] * col[jj];
            }
        }
        __syncthreads();
        if (fail) continue;  // recompute S, then pseudo-inverse
        // X = L^-1 (row-major lower), column by column of the identity
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
            const int i = idx / na, j = idx - (idx / na) * na;
            X[idx] = (i == j) ? 1.0 : 0.0;
        }
        for (int k = 0; k < na; ++k) {
            __syncthreads();
            const double inv = 1.0 / S[(size_t)k * na + k];
            for (int j = threadIdx.x; j <= k; j += blockDim.x) X[(size_t)k * na + j] *= inv;
            __syncthreads();
            const int w = na - k - 1;
            for (int idx = threadIdx.x; idx < w * (k + 1); idx += blockDim.x) {
                const int i = k + 1 + idx / (k + 1), j = idx - (idx / (k + 1)) * (k + 1);
                X[(size_t)i * na + j] -= S[(size_t)i * na + k] * X[(size_t)k * na + j];
            }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
            const int i = idx / na, j = idx - (idx / na) * na;
            double s = 0.0;
            for (int k = (i > j ? i : j); k < na; ++k)
                s += X[(size_t)k * na + i] * X[(size_t)k * na + j];
            G[idx] = s;
        }
        return;
    }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
    return s;
}

__global__ __launch_bounds__(256) void pc_apply1_kernel(
    int N, const int *__restrict__ blob_off, const int64_t *__restrict__ mat_off,
    const int64_t *__restrict__ z_off, const double *__restrict__ minv,
    const double *__restrict__ Zbuf, const double *__restrict__ Nt, const double *__restrict__ r,
    double *__restrict__ z, double *__restrict__ uhat) {
    __shared__ double x[kMaxM];
    __shared__ double red[8];
    __shared__ double w6[6];
    const int p = blockIdx.x;
    const int b0 = blob_off[p], m = 3 * (blob_off[p + 1] - b0);
    const double *Mi = minv + mat_off[p];
    const double *Z = Zbuf + z_off[p];
    const double *rl = r + 3 * (size_t)b0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) x[i] = rl[i];
    __syncthreads();
    // t = Minv r_lam (Minv symmetric: column access is coalesced)
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Mi[(size_t)k * m + i] * x[k];
        z[3 * (size_t)b0 + i] = s;
    }
    // Z^T r_lam
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        for (int c = 0; c < 6; ++c) acc[c] += Z[(size_t)i * 6 + c] * x[i];
    for (int c = 0; c < 6; ++c) {
        const double s = block_sum(acc[c], red);
        if (threadIdx.x == 0) w6[c] = s + r[3 * (size_t)N + 6 * (size_t)p + c];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double *Nb = Nt + 36 * (size_t)p;
        double s = 0.0;
        for (int c = 0; c < 6; ++c) s += Nb[threadIdx.x * 6 + c] * w6[c];
        uhat[6 * (size_t)p + threadIdx.x] = -s;
    }
}

__global__ __launch_bounds__(256) void pc_apply2_kernel(
    int N, int M, const int *__restrict__ asm_row_ptr, const int *__restrict__ asm_rows,
    const int64_t *__restrict__ asm_mat_off, const int *__restrict__ row_p,
    const int *__restrict__ row_q, const double *__restrict__ crow, const double *__restrict__ Gbuf,
    const double *__restrict__ r, const double *__restrict__ uhat, double *__restrict__ z) {
    __shared__ double y[kMaxAsmRows];
    const int a = blockIdx.x;
    const int r0 = asm_row_ptr[a], na = asm_row_ptr[a + 1] - r0;
    if (na == 0) return;
    const double *G = Gbuf + asm_mat_off[a];
    const size_t off_phi = 3 * (size_t)N + 6 * (size_t)M;
    for (int k = threadIdx.x; k < na; k += blockDim.x) {
        const int rk = asm_rows[r0 + k];
        const double *c = crow + 12 * (size_t)rk;
        const double *Up = uhat + 6 * (size_t)row_p[rk];
        double s = 0.0;
        for (int u = 0; u < 6; ++u) s += c[u] * Up[u];
        const int q = row_q[rk];
        if (q >= 0) {
            const double *Uq = uhat + 6 * (size_t)q;
            for (int u = 0; u < 6; ++u) s += c[6 + u] * Uq[u];
        }
        y[k] = r[off_phi + rk] - s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < na; k += blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < na; ++l) s += G[(size_t)k * na + l] * y[l];
        z[off_phi + asm_rows[r0 + k]] = s;
    }
}

__global__ __launch_bounds__(256) void pc_apply3_kernel(
    int N, int M, const int *__restrict__ blob_off, const int64_t *__restrict__ z_off,
    const double *__restrict__ Zbuf, const double *__restrict__ Nt,
    const int *__restrict__ brow_ptr, const int *__restrict__ brow_ent,
    const double *__restrict__ crow, const double *__restrict__ uhat, double *__restrict__ z,
    int has_rows) {
    __shared__ double U[6];
    __shared__ double f[6];
    const int p = blockIdx.x;
    const size_t off_phi = 3 * (size_t)N + 6 * (size_t)M;
    if (threadIdx.x < 6) {
        double s = 0.0;
        if (has_rows) {
            for (int e = brow_ptr[p]; e < brow_ptr[p + 1]; ++e) {
                const int ent = brow_ent[e];
                const int row = ent >> 1, side = ent & 1;
                s += z[off_phi + row] * crow[12 * (size_t)row + 6 * side + threadIdx.x];
            }
        }
        f[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double *Nb = Nt + 36 * (size_t)p;
        double s = uhat[6 * (size_t)p + threadIdx.x];
        for (int c = 0; c < 6; ++c) s += Nb[threadIdx.x * 6 + c] * f[c];
        U[threadIdx.x] = s;
        z[3 * (size_t)N + 6 * (size_t)p + threadIdx.x] = s;
    }
    __syncthreads();
    const int b0 = blob_off[p], m = 3 * (blob_off[p + 1] - b0);
    const double *Z = Zbuf + z_off[p];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < 6; ++c) s += Z[(size_t)i * 6 + c] * U[c];
        z[3 * (size_t)b0 + i] += s;
    }
}


// Per-type variants (learned body mobility and body-frame blocks): each body's
// block starts from the unbounded blob mobility of its type in the body frame
// (factored once), rotated by R_p: A_p = (I x R) Minv_type (I x R^T),
// Z_f = A_p K_p = (I x R) Z_type Q^T with Q = diag(R, R), N~_f = Q N~_type Q^T.
// Body-frame variant: N~_p = N~_f, an exact block solve of the unbounded blocks.
// Learned variant: the network gives the wall body mobility N~_w, and the blob
// block is modified by a rank-6 term so that the block solve stays exact for
// a consistent pair (M~, N~_w):
//   M~^-1 = A_p + Z_f D Z_f^T,  D = N~_f N~_w^-1 N~_f - N~_f,
// which gives K^T M~^-1 K = N~_w^-1 and K^T M~^-1 = N~_w^-1 N~_f Z_f^T.  Per body
// E1 = D and E2 = D N~_f^-1 are formed at build time; the apply then reads
//   U^ = -N~_w r_U - N~_f s,  s = Z_f^T r_lam,
//   lam = A_p r_lam + Z_f (U + E1 s + E2 U),
// with U = U^ + N~_w C^T phi as in the exact variant.
__global__ __launch_bounds__(256) void pc_apply1_learned_kernel(
    int N, const int *__restrict__ blob_off, const int *__restrict__ type,
    const int64_t *__restrict__ tmat_off, const int64_t *__restrict__ tz_off,
    const double *__restrict__ tminv, const double *__restrict__ tZ, const double *__restrict__ R9,
    const double *__restrict__ Nt, const double *__restrict__ lcorr, const double *__restrict__ r,
    double *__restrict__ z, double *__restrict__ uhat, double *__restrict__ stmp) {
    __shared__ double x[kMaxM];
    __shared__ double tb[kMaxM];
    __shared__ double red[8];
    __shared__ double w6[6];
    __shared__ double R[9];
    const int p = blockIdx.x;
    const int b0 = blob_off[p], n = blob_off[p + 1] - b0, m = 3 * n;
    const int ty = type[p];
    const double *Mi = tminv + tmat_off[ty];
    const double *Z = tZ + tz_off[ty];
    if (threadIdx.x < 9) R[threadIdx.x] = R9[9 * (size_t)p + threadIdx.x];
    __syncthreads();
    const double *rl = r + 3 * (size_t)b0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // x_b = R^T r_lam (per blob)
        const double a0 = rl[3 * i], a1 = rl[3 * i + 1], a2 = rl[3 * i + 2];
        for (int c = 0; c < 3; ++c) x[3 * i + c] = R[c] * a0 + R[3 + c] * a1 + R[6 + c] * a2;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Mi[(size_t)k * m + i] * x[k];
        tb[i] = s;
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < m; i += blockDim.x)
        for (int c = 0; c < 6; ++c) acc[c] += Z[(size_t)i * 6 + c] * x[i];
    double zb[6];
    for (int c = 0; c < 6; ++c) zb[c] = block_sum(acc[c], red);  // syncs: tb complete
    for (int i = threadIdx.x; i < n; i += blockDim.x) {  // t_p = R t_b
        const double a0 = tb[3 * i], a1 = tb[3 * i + 1], a2 = tb[3 * i + 2];
        for (int c = 0; c < 3; ++c)
            z[3 * (size_t)b0 + 3 * i + c] = R[3 * c] * a0 + R[3 * c + 1] * a1 + R[3 * c + 2] * a2;
    }
    __shared__ double s6[6];
    if (threadIdx.x < 6) {
        // s = Z_f^T r_lam = Q (Z_type^T x_b)
        const int h = threadIdx.x / 3, c = threadIdx.x % 3;
        const double v = R[3 * c] * zb[3 * h] + R[3 * c + 1] * zb[3 * h + 1] + R[3 * c + 2] * zb[3 * h + 2];
        const double ru = r[3 * (size_t)N + 6 * (size_t)p + threadIdx.x];
        s6[threadIdx.x] = v;
        w6[threadIdx.x] = lcorr ? ru : v + ru;
        if (lcorr) stmp[6 * (size_t)p + threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double *Nb = Nt + 36 * (size_t)p;
        double acc = 0.0;
        for (int c = 0; c < 6; ++c) acc += Nb[threadIdx.x * 6 + c] * w6[c];
        if (lcorr) {  // - N~_f s
            const double *Nf = lcorr + 108 * (size_t)p;
            for (int c = 0; c < 6; ++c) acc += Nf[threadIdx.x * 6 + c] * s6[c];
        }
        uhat[6 * (size_t)p + threadIdx.x] = -acc;
    }
}

__global__ __launch_bounds__(256) void pc_apply3_learned_kernel(
    int N, int M, const int *__restrict__ blob_off, const int *__restrict__ type,
    const int64_t *__restrict__ tz_off, const double *__restrict__ tZ, const double *__restrict__ R9,
    const double *__restrict__ Nt, const double *__restrict__ lcorr,
    const double *__restrict__ stmp, const int *__restrict__ brow_ptr,
    const int *__restrict__ brow_ent, const double *__restrict__ crow,
    const double *__restrict__ uhat, double *__restrict__ z, int has_rows) {
    __shared__ double U[6], V[6], Ub[6], f[6], R[9];
    const int p = blockIdx.x;
    const size_t off_phi = 3 * (size_t)N + 6 * (size_t)M;
    if (threadIdx.x < 9) R[threadIdx.x] = R9[9 * (size_t)p + threadIdx.x];
    if (threadIdx.x < 6) {
        double s = 0.0;
        if (has_rows) {
            for (int e = brow_ptr[p]; e < brow_ptr[p + 1]; ++e) {
                const int ent = brow_ent[e];
                const int row = ent >> 1, side = ent & 1;
                s += z[off_phi + row] * crow[12 * (size_t)row + 6 * side + threadIdx.x];
            }
        }
        f[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double *Nb = Nt + 36 * (size_t)p;
        double s = uhat[6 * (size_t)p + threadIdx.x];
        for (int c = 0; c < 6; ++c) s += Nb[threadIdx.x * 6 + c] * f[c];
        U[threadIdx.x] = s;
        z[3 * (size_t)N + 6 * (size_t)p + threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {  // V = U (+ E1 s + E2 U with the learned correction)
        double v = U[threadIdx.x];
        if (lcorr) {
            const double *E1 = lcorr + 108 * (size_t)p + 36, *E2 = E1 + 36;
            const double *sp = stmp + 6 * (size_t)p;
            for (int c = 0; c < 6; ++c) v += E1[threadIdx.x * 6 + c] * sp[c] + E2[threadIdx.x * 6 + c] * U[c];
        }
        V[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {  // Q^T V
        const int h = threadIdx.x / 3, c = threadIdx.x % 3;
        Ub[threadIdx.x] = R[c] * V[3 * h] + R[3 + c] * V[3 * h + 1] + R[6 + c] * V[3 * h + 2];
    }
    __syncthreads();
    const int b0 = blob_off[p], n = blob_off[p + 1] - b0;
    const double *Z = tZ + tz_off[type[p]];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v[3];
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += Z[(size_t)(3 * i + c) * 6 + k] * Ub[k];
            v[c] = s;
        }
        for (int c = 0; c < 3; ++c)
            z[3 * (size_t)b0 + 3 * i + c] += R[3 * c] * v[0] + R[3 * c + 1] * v[1] + R[3 * c + 2] * v[2];
    }
}

// N~_p = Q N~_type Q^T, Q = diag(R_p, R_p): the free-space body mobility of
// the body's type rotated into its orientation (no wall)
__global__ void pc_rotate_nt_kernel(int M, const int *__restrict__ type,
                                    const double *__restrict__ tNt, const double *__restrict__ R9,
                                    double *__restrict__ Nt) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double *R = R9 + 9 * (size_t)p;
    const double *A = tNt + 36 * (size_t)type[p];
    double T[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {  // (Q A)_ij
            const int bi = i / 3, ri = i % 3;
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += R[3 * ri + k] * A[(3 * bi + k) * 6 + j];
            T[i * 6 + j] = s;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {  // (Q A) Q^T
            const int bj = j / 3, rj = j % 3;
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[i * 6 + 3 * bj + k] * R[3 * rj + k];
            Nt[36 * (size_t)p + i * 6 + j] = s;
        }
}

// 6 x 6 SPD inverse by Cholesky; false if a pivot is not positive
__device__ bool spd6_inverse(const double *A, double *X) {
    double L[36] = {};
    for (int j = 0; j < 6; ++j) {
        double d = A[j * 6 + j];
        for (int k = 0; k < j; ++k) d -= L[j * 6 + k] * L[j * 6 + k];
        if (!(d > 0.0)) return false;
        L[j * 6 + j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = 0.5 * (A[i * 6 + j] + A[j * 6 + i]);
            for (int k = 0; k < j; ++k) v -= L[i * 6 + k] * L[j * 6 + k];
            L[i * 6 + j] = v / L[j * 6 + j];
        }
    }
    for (int c = 0; c < 6; ++c) {  // X e_c = L^-T L^-1 e_c
        double y[6];
        for (int i = 0; i < 6; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[i * 6 + k] * y[k];
            y[i] = v / L[i * 6 + i];
        }
        for (int i = 5; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < 6; ++k) v -= L[k * 6 + i] * y[k];
            y[i] = v / L[i * 6 + i];
        }
        for (int i = 0; i < 6; ++i) X[i * 6 + c] = y[i];
    }
    return true;
}

// per body: N~_f (rotated type mobility), E1 = N~_f N~_w^-1 N~_f - N~_f,
// E2 = E1 N~_f^-1 (108 doubles); flags bodies whose N~_w or N~_f is not SPD
__global__ void pc_learned_corr_kernel(int M, const int *__restrict__ type,
                                       const double *__restrict__ tNt,
                                       const double *__restrict__ R9,
                                       const double *__restrict__ Nw, double *__restrict__ out,
                                       int *__restrict__ bad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double *R = R9 + 9 * (size_t)p;
    const double *A = tNt + 36 * (size_t)type[p];
    double T[36], Nf[36], Wi[36], Fi[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const int bi = i / 3, ri = i % 3;
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += R[3 * ri + k] * A[(3 * bi + k) * 6 + j];
            T[i * 6 + j] = s;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const int bj = j / 3, rj = j % 3;
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[i * 6 + 3 * bj + k] * R[3 * rj + k];
            Nf[i * 6 + j] = s;
        }
    const bool ok = spd6_inverse(Nw + 36 * (size_t)p, Wi) && spd6_inverse(Nf, Fi);
    if (!ok) atomicOr(bad, 1);
    double *o = out + 108 * (size_t)p;
    for (int k = 0; k < 36; ++k) o[k] = Nf[k];
    double WN[36], E1[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += Wi[i * 6 + k] * Nf[k * 6 + j];
            WN[i * 6 + j] = s;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = -Nf[i * 6 + j];
            for (int k = 0; k < 6; ++k) s += Nf[i * 6 + k] * WN[k * 6 + j];
            E1[i * 6 + j] = ok ? s : 0.0;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += E1[i * 6 + k] * Fi[k * 6 + j];
            o[36 + i * 6 + j] = E1[i * 6 + j];
            o[72 + i * 6 + j] = ok ? s : 0.0;
        }
}

void learned_correction(hipStream_t s, int M, const int *type, const double *tNt,
                        const double *R9, const double *Nw, double *out, int *bad) {
    if (M > 0)
        pc_learned_corr_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, type, tNt, R9, Nw, out, bad);
}

void rotate_body_mobility(hipStream_t s, int M, const int *type, const double *tNt,
                          const double *R9, double *Nt) {
    if (M > 0) pc_rotate_nt_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, type, tNt, R9, Nt);
}

void precond_assemble(hipStream_t s, const PrecondDev &P, const double *pos, double a, double eta,
                      bool wall) {
    if (P.M <= 0) return;
    const CoefD c = make_coef<CoefD, double>(a);
    pc_assemble_kernel<<<P.M, 256, 0, s>>>(P.blob_off, P.mat_off, pos, c, 1.0 / (8 * kPi * eta),
                                           wall ? 1 : 0, a, P.mats, P.status);
}

// SPD inverse of each matrix of the batch by the symmetric block sweep (block
// Gauss-Jordan elimination without pivoting, which positive definite matrices
// allow; the pivot blocks are the Schur complements of the Cholesky
// factorisation), out of place, for matrices of at most kSwRows rows.  One
// workgroup of 512 threads per matrix holds its lower triangle in registers as
// 16 x 16 tiles in the matrix-core accumulator layout: tile t = (ti, tj), tj <= ti,
// counted row by row, belongs to wavefront t % 8 (slot t / 8).  Rows beyond m
// are padded with the identity.  Sweeping block k with P = A_kk^-1 takes, with
// the values before the step,
//   A_ij -= A_ik P A_kj (i, j != k),   A_ik <- A_ik P,   A_kk <- -P,
// which keeps the matrix symmetric; after the last block it holds -A^-1.  Per
// step: the block column k is copied to LDS (C_r = A_rk, the tiles of row k
// transposed); one wavefront inverts D = A_kk in place there by Gauss-Jordan
// steps, testing each pivot (the Cholesky pivots, L_ii^2)
// against rel_tol * (largest diagonal entry) as pc_potrf does and storing
// sqrt(pivot) as diag(L) when asked; W_r = C_r P is formed on the matrix cores
// (wavefront r % 8 takes block row r); every wavefront then updates its tiles on the
// matrix cores, A_ij -= W_i C_j^T.  The flop count equals that of factor,
// triangular inverse and product (m^3 in all), with the matrix read once and
// its inverse (both triangles) written once.  Dynamic LDS: C and W, 16 nb rows
// of kSwLd doubles each.
constexpr int kSwRows = 256;
constexpr int kSwThreads = 512;
constexpr int kSwWaves = kSwThreads / 64;
constexpr int kSwLd = 17;
// matrices of at most kSwSmall tile rows (144 rows) take an instance with fewer
// registers, two or more workgroups per compute unit
constexpr int kSwSmall = 9;

size_t sweep_lds_bytes(int max_m) {
    const int nb = (max_m + 15) / 16;
    return 2 * (size_t)16 * nb * kSwLd * sizeof(double);
}

// NBMAX: the most tile rows this instance holds; matrices of at most nb_lo tile
// rows (or more than NBMAX) are skipped
template <int NBMAX>
__global__ __launch_bounds__(kSwThreads) void pc_sweep_kernel(MatBatch B, int nb_lo) {
    constexpr int kSwSlots = (NBMAX * (NBMAX + 1) / 2 + kSwWaves - 1) / kSwWaves;
    extern __shared__ double sw_lds[];
    __shared__ int fail;
    __shared__ double piv_tol;
    __shared__ double red[kSwWaves];
    const int p = blockIdx.x;
    if (mat_skip(B, p)) return;
    const int m = mat_rows(B, p);
    const int nb = (m + 15) >> 4, T = nb * (nb + 1) / 2;
    if (nb <= nb_lo || nb > NBMAX) return;
    double *Cb = sw_lds;                            // C_r = A_rk, 16 nb x kSwLd
    double *Wb = sw_lds + (size_t)16 * nb * kSwLd;  // W_r = C_r P
    const double *A = B.mats + B.mat_off[p];
    double *Out = B.out + B.mat_off[p];
    const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // this wavefront's tiles: row i of tile t is the largest with i (i + 1) / 2 <= t
    int ti[kSwSlots], tj[kSwSlots];
#pragma unroll
    for (int s = 0; s < kSwSlots; ++s) {
        const int t = w + kSwWaves * s;
        int i = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
        i += (i + 1) * (i + 2) / 2 <= t;
        i -= i * (i + 1) / 2 > t;
        ti[s] = i;
        tj[s] = t - i * (i + 1) / 2;
    }
    // load the lower triangle (the upper part of diagonal tiles by symmetry)
    mfma_acc acc[kSwSlots];
    double dloc = 0.0;
#pragma unroll
    for (int s = 0; s < kSwSlots; ++s) {
        if (w + kSwWaves * s >= T) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * ti[s] + 4 * e + lr, c = 16 * tj[s] + lc;
            double v = r == c ? 1.0 : 0.0;
            if (r < m && c < m) v = c <= r ? A[(size_t)r * m + c] : A[(size_t)c * m + r];
            acc[s][e] = v;
            if (r == c && r < m) dloc = fmax(dloc, v);
        }
    }
    if (B.rel_tol > 0.0) {
        for (int o = 32; o > 0; o >>= 1) dloc = fmax(dloc, __shfl_xor(dloc, o));
        if (l == 0) red[w] = dloc;
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    if (tid == 0) {
        double dmax = 0.0;
        if (B.rel_tol > 0.0)
            for (int q = 0; q < kSwWaves; ++q) dmax = fmax(dmax, red[q]);
        piv_tol = B.rel_tol * dmax;
    }
    for (int k = 0; k < nb; ++k) {
        double *Dk = Cb + (size_t)16 * k * kSwLd;  // rows of C holding D = A_kk, then P
        __syncthreads();  // the previous step's reads of C and W are done
        // 1. block column k: C_r = A_rk (tiles (r, k), r >= k, and (k, r)^T, r < k)
#pragma unroll
        for (int s = 0; s < kSwSlots; ++s) {
            if (w + kSwWaves * s >= T) continue;
            if (tj[s] == k) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Cb[(16 * ti[s] + 4 * e + lr) * kSwLd + lc] = acc[s][e];
            } else if (ti[s] == k) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Cb[(16 * tj[s] + lc) * kSwLd + 4 * e + lr] = acc[s][e];
            }
        }
        __syncthreads();
        // 2. P = D^-1 by Gauss-Jordan in wavefront 0, in place in the LDS rows of C
        // that hold D (no later use of C_k): lane l keeps D[4e + l/16][l%16] in
        // registers and publishes it after every pivot; one wavefront's LDS
        // operations complete in order, so each pivot reads the previous one's
        // values (the fences keep the compiler from reordering them)
        if (w == 0) {
            const double tol = piv_tol;
            double d[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) d[e] = Dk[(4 * e + lr) * kSwLd + lc];
            bool bad = false;
            double mypiv = 1.0;  // lane q < 16: pivot q
#pragma unroll 1
            for (int q = 0; q < 16; ++q) {
                const double piv = Dk[q * kSwLd + q];
                const double rqc = Dk[q * kSwLd + lc];  // D_q,c
                double cq[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) cq[e] = Dk[(4 * e + lr) * kSwLd + q];  // D_r,q
                // a failed pivot is recorded, the (meaningless) steps still run
                bad |= !(piv > tol);
                mypiv = l == q ? piv : mypiv;
                // 1 / piv: the hardware estimate and two Newton steps
                double ip = __builtin_amdgcn_rcp(piv);
                ip = fma(fma(-piv, ip, 1.0), ip, ip);
                ip = fma(fma(-piv, ip, 1.0), ip, ip);
                const double rq = rqc * ip;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // pivot row scaled, pivot column scaled and negated, the rest
                    // eliminated; selects, no branches
                    const bool rowq = 4 * e + lr == q, colq = lc == q;
                    const double sc = d[e] * ip, el = fma(-cq[e], rq, d[e]);
                    d[e] = rowq ? (colq ? ip : sc) : (colq ? -sc : el);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
                for (int e = 0; e < 4; ++e) Dk[(4 * e + lr) * kSwLd + lc] = d[e];
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (B.ldiag && l < 16 && 16 * k + l < m)
                B.ldiag[B.scale * (int64_t)B.off[p] + 16 * k + l] = sqrt(mypiv);
            if (bad && l == 0) fail = 1;
        }
        __syncthreads();
        if (fail) break;
        // 3. W_r = C_r P, block row r by wavefront r % kSwWaves
        for (int r = w; r < nb; r += kSwWaves) {
            if (r == k) continue;
            mfma_acc x = {};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                x = mfma_f64_16x16x4(Cb[(16 * r + lc) * kSwLd + 4 * kk + lr],
                                     Dk[(4 * kk + lr) * kSwLd + lc], x);
#pragma unroll
            for (int e = 0; e < 4; ++e) Wb[(16 * r + 4 * e + lr) * kSwLd + lc] = x[e];
        }
        __syncthreads();
        // 4. the tiles: A_ij -= W_i C_j^T; A_ik <- W_i; A_kj <- W_j^T; A_kk <- -P
#pragma unroll
        for (int s = 0; s < kSwSlots; ++s) {
            if (w + kSwWaves * s >= T) continue;
            const int i = ti[s], j = tj[s];
            if (i != k && j != k) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    acc[s] = mfma_f64_16x16x4(-Wb[(16 * i + lc) * kSwLd + 4 * kk + lr],
                                              Cb[(16 * j + lc) * kSwLd + 4 * kk + lr], acc[s]);
            } else if (i != k) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[s][e] = Wb[(16 * i + 4 * e + lr) * kSwLd + lc];
            } else if (j != k) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[s][e] = Wb[(16 * j + lc) * kSwLd + 4 * e + lr];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[s][e] = -Dk[(4 * e + lr) * kSwLd + lc];
            }
        }
    }
    if (fail) {
        if (tid == 0) {
            if (B.fail)
                B.fail[p] = 1;
            else
                atomicMax(&B.status[0], p + 1);
        }
        return;
    }
    // A^-1 = -(the tiles), both triangles
#pragma unroll
    for (int s = 0; s < kSwSlots; ++s) {
        if (w + kSwWaves * s >= T) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * ti[s] + 4 * e + lr, c = 16 * tj[s] + lc;
            if (r < m && c < m) {
                Out[(size_t)r * m + c] = -acc[s][e];
                if (ti[s] != tj[s]) Out[(size_t)c * m + r] = -acc[s][e];
            }
        }
    }
}

bool precond_factor_in_place(int max_m) { return max_m > kSwRows; }

// the sweep over a batch of count matrices of at most max_m <= kSwRows rows: the
// small instance when every matrix fits it, else the large one for all of them
// (one launch keeps small and large matrices interleaved over the compute units;
// two launches measured slower on the bacteria)
static hipError_t launch_sweep(hipStream_t s, const MatBatch &B, int count, int max_m) {
    const size_t lds = sweep_lds_bytes(max_m);
    if (max_m <= 16 * kSwSmall) {
        const hipError_t e = hipFuncSetAttribute((const void *)pc_sweep_kernel<kSwSmall>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
        pc_sweep_kernel<kSwSmall><<<count, kSwThreads, lds, s>>>(B, 0);
    } else {
        const hipError_t e = hipFuncSetAttribute((const void *)pc_sweep_kernel<kSwRows / 16>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
        pc_sweep_kernel<kSwRows / 16><<<count, kSwThreads, lds, s>>>(B, 0);
    }
    return hipSuccess;
}

hipError_t precond_factor(hipStream_t s, const PrecondDev &P, const double *dvec, int max_m) {
    if (P.M <= 0) return hipSuccess;
    if (max_m <= kSwRows) {
        const MatBatch B{P.blob_off, 3, P.mat_off, P.mats, P.ldiag, P.dinv, P.minv, P.status,
                         nullptr, 0.0};
        const hipError_t e = launch_sweep(s, B, P.M, max_m);
        if (e != hipSuccess) return e;
    } else if (max_m <= kFastMaxM) {
        const int nbk = (max_m + kNB - 1) / kNB;
        const size_t lds_i = (size_t)nbk * kNB * kLd * sizeof(double);
        const hipError_t e = hipFuncSetAttribute(
            (const void *)pc_trtri_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_i);
        if (e != hipSuccess) return e;
        const int nt = (max_m + 63) / 64;
        const MatBatch B{P.blob_off, 3, P.mat_off, P.mats, P.ldiag, P.dinv, P.minv, P.status,
                         nullptr, 0.0};
        pc_potrf_kernel<<<P.M, 256, 0, s>>>(B);
        pc_trtri_kernel<<<dim3(nbk, P.M), 256, lds_i, s>>>(B);
        pc_lauum_kernel<<<dim3(nt * (nt + 1) / 2, P.M), 256, 0, s>>>(B);
    } else {
        pc_chol_kernel<<<P.M, 256, 0, s>>>(P.blob_off, P.mat_off, P.mats, P.ldiag, P.status);
        pc_inverse_kernel<<<P.M, 256, 0, s>>>(P.blob_off, P.mat_off, P.mats, P.ldiag, P.minv,
                                              P.status);
        pc_restore_diag_kernel<<<P.M, 256, 0, s>>>(P.blob_off, P.mat_off, P.mats, P.ldiag);
    }
    pc_body_kernel<<<P.M, 256, 0, s>>>(P.blob_off, P.mat_off, P.z_off, P.minv, dvec, P.Z, P.Nt,
                                       P.body_pinv, P.status);
    pc_body_pinv_kernel<<<(P.M + 63) / 64, 64, 0, s>>>(P.M, P.body_pinv, P.Nt, P.status);
    return hipGetLastError();
}

// doubles needed for the diagonal-block inverses of bodies holding n_blobs blobs
int64_t precond_dinv_size(int64_t n_blobs, int M) { return 32 * 3 * n_blobs + 1024 * (int64_t)M; }

// Single-blob bodies (Sec. 2.4 with Sec. 3.1): N~_p = diag(mt I, mr I), the
// self mobilities 1/(6 pi eta a) and 1/(8 pi eta a^3)
__global__ void single_blob_nt_kernel(int M, double mt, double mr, double *__restrict__ Nt) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 36 * M) return;
    const int e = idx % 36, r = e / 6, c = e % 6;
    Nt[idx] = r != c ? 0.0 : (r < 3 ? mt : mr);
}

__global__ void copy_kernel(int64_t n, const double *__restrict__ x, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

void single_blob_body_mobility(hipStream_t s, int M, double a, double eta, double *Nt) {
    if (M <= 0) return;
    single_blob_nt_kernel<<<(36 * M + 255) / 256, 256, 0, s>>>(
        M, 1.0 / (6.0 * kPi * eta * a), 1.0 / (8.0 * kPi * eta * a * a * a), Nt);
}

// z = P^-1 r for y = [U; phi]: phi = G~ (r_phi - C r_U), U = r_U + N~ C^T phi.
// These are the assembly and body stages of the multiblob apply with no blobs
// (r_U takes the place of U^); zero_off / zero_off64 are M+1 zeros.
void precond_apply_single(hipStream_t s, const PrecondDev &P, const int *zero_off,
                          const int64_t *zero_off64, const double *r, double *z) {
    if (P.M <= 0) return;
    const int64_t m6 = 6 * (int64_t)P.M;
    copy_kernel<<<(int)((m6 + 255) / 256), 256, 0, s>>>(m6, r, P.tmp);
    if (P.A > 0)
        pc_apply2_kernel<<<P.A, 256, 0, s>>>(0, P.M, P.asm_row_ptr, P.asm_rows, P.asm_mat_off,
                                             P.row_p, P.row_q, P.crow, P.G, r, P.tmp, z);
    pc_apply3_kernel<<<P.M, 256, 0, s>>>(0, P.M, zero_off, zero_off64, P.Nt, P.Nt, P.brow_ptr,
                                         P.brow_ent, P.crow, P.tmp, z, P.A > 0 ? 1 : 0);
}

// G~_a = S_a^-1 for every assembly (Sec. 3.1), with a pivot test relative to the
// largest diagonal entry; assemblies that fail it (constraints without full row
// rank) take the symmetric pseudo-inverse.  Largest assembly of at most kAsmSmall
// rows: one workgroup per assembly in LDS; up to kFastMaxM rows: the blocked
// kernels of the blob mobilities (S_a formed in P.S, factored in place, the
// inverse written to P.G); beyond: the unblocked kernel.
hipError_t precond_assembly(hipStream_t s, const PrecondDev &P) {
    if (P.A <= 0) return hipSuccess;
    const int nmax = std::max(P.asm_max_rows, 1);
    if (nmax <= kAsmSmall && P.asm_fail) {
        const size_t lds = (2 * (size_t)nmax * (nmax + 1) + 24 * (size_t)nmax) * sizeof(double) +
                           2 * (size_t)nmax * sizeof(int);
        const hipError_t e = hipFuncSetAttribute(
            (const void *)pc_asm_small_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        pc_asm_small_kernel<<<P.A, kAsmThreads, lds, s>>>(P.asm_row_ptr, P.asm_rows,
                                                          P.asm_mat_off, P.row_p, P.row_q, P.crow,
                                                          P.Nt, P.G, P.asm_fail, P.status, nmax);
        pc_asm_pinv_kernel<<<P.A, 256, 0, s>>>(P.asm_row_ptr, P.asm_rows, P.asm_mat_off, P.row_p,
                                               P.row_q, P.crow, P.Nt, P.S, P.G, P.asm_fail,
                                               P.status);
        return hipGetLastError();
    }
    if (P.asm_max_rows > kFastMaxM || !P.asm_dinv || !P.asm_fail) {
        pc_asm_kernel<<<P.A, 256, 0, s>>>(P.asm_row_ptr, P.asm_rows, P.asm_mat_off, P.row_p,
                                          P.row_q, P.crow, P.Nt, P.S, P.G, P.status);
        return hipGetLastError();
    }
    const int max_m = nmax;
    const int nbk = (max_m + kNB - 1) / kNB;
    const size_t lds_i = (size_t)nbk * kNB * kLd * sizeof(double);
    const size_t lds_r = 12 * (size_t)max_m * sizeof(double) + 2 * (size_t)max_m * sizeof(int);
    const bool sweep = max_m <= kSwRows;
    hipError_t e = hipFuncSetAttribute((const void *)pc_trtri_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_i);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)pc_asm_form_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_r);
    if (e != hipSuccess) return e;
    const int nt = (max_m + 63) / 64;
    pc_asm_form_kernel<<<P.A, 256, lds_r, s>>>(P.asm_row_ptr, P.asm_rows, P.asm_mat_off,
                                               P.row_p, P.row_q, P.crow, P.Nt, P.S, P.asm_fail,
                                               P.status, max_m);
    const MatBatch B{P.asm_row_ptr, 1, P.asm_mat_off, P.S, nullptr, P.asm_dinv, P.G, P.status,
                     P.asm_fail, 1e-12};
    if (sweep) {
        e = launch_sweep(s, B, P.A, max_m);
        if (e != hipSuccess) return e;
    } else {
        pc_potrf_kernel<<<P.A, 256, 0, s>>>(B);
        pc_trtri_kernel<<<dim3(nbk, P.A), 256, lds_i, s>>>(B);
        pc_lauum_kernel<<<dim3(nt * (nt + 1) / 2, P.A), 256, 0, s>>>(B);
    }
    pc_asm_pinv_kernel<<<P.A, 256, 0, s>>>(P.asm_row_ptr, P.asm_rows, P.asm_mat_off, P.row_p,
                                           P.row_q, P.crow, P.Nt, P.S, P.G, P.asm_fail, P.status);
    return hipGetLastError();
}

void precond_apply(hipStream_t s, const PrecondDev &P, int N, const double *r, double *z) {
    if (P.M <= 0) return;
    if (P.learned)
        pc_apply1_learned_kernel<<<P.M, 256, 0, s>>>(N, P.blob_off, P.type, P.tmat_off, P.tz_off,
                                                     P.tminv, P.tZ, P.R9, P.Nt, P.lcorr, r, z,
                                                     P.tmp, P.stmp);
    else
        pc_apply1_kernel<<<P.M, 256, 0, s>>>(N, P.blob_off, P.mat_off, P.z_off, P.minv, P.Z, P.Nt,
                                             r, z, P.tmp);
    if (P.A > 0)
        pc_apply2_kernel<<<P.A, 256, 0, s>>>(N, P.M, P.asm_row_ptr, P.asm_rows, P.asm_mat_off,
                                             P.row_p, P.row_q, P.crow, P.G, r, P.tmp, z);
    if (P.learned)
        pc_apply3_learned_kernel<<<P.M, 256, 0, s>>>(N, P.M, P.blob_off, P.type, P.tz_off, P.tZ,
                                                     P.R9, P.Nt, P.lcorr, P.stmp, P.brow_ptr,
                                                     P.brow_ent, P.crow, P.tmp, z,
                                                     P.A > 0 ? 1 : 0);
    else
        pc_apply3_kernel<<<P.M, 256, 0, s>>>(N, P.M, P.blob_off, P.z_off, P.Z, P.Nt, P.brow_ptr,
                                             P.brow_ent, P.crow, P.tmp, z, P.A > 0 ? 1 : 0);
}

}  // namespace arb
