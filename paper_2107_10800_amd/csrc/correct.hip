// Position/orientation correction (Sec. 4.2, Eq. min_probl / Eq. residual, App. B).
//
// One workgroup per articulated body (bodies joined by links).  Unknowns per
// body: dq (3) and a quaternion dtheta (4), starting at (0, [1,0,0,0]).
// Residuals: g_n = q_p + dq_p + R(dtheta_p) l~_p - q_q - dq_q - R(dtheta_q) l~_q
// with l~ = R(theta) dl (App. B form), plus ||dtheta_p||^2 - 1 per body.
// Jacobian from Eq. rot_mat: dg/ddq = I, dg/ds = 2 p x l~ + 4 s l~,
// dg_i/dp_l = 2 [delta_il (p.l~) + p_i l~_l + s eps_ilk l~_k]  (30 non-zeros per link).
// Levenberg-Marquardt with mu = ||F||^2: delta = -J^T (J J^T + mu I)^-1 F,
// accepted if ||F|| decreases, else mu *= 10 (at most 20 tries); stop at
// ||F|| <= tol or max_iter accepted steps.  Then dtheta is normalised and
// q <- q + dq, theta <- dtheta . theta (Sec. 4.3 step 5).
// All loops are bounded; every thread follows the same control flow.
#include "common.h"

namespace arb {

constexpr int kMaxCorrRows = 2048;

__device__ __forceinline__ double block_sum_c(double v, double *red) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += red[k];
    return s;
}

// workspace layout per assembly (doubles):
//   lt [6 nl] | x [7 nb] | xn [7 nb] | F [nF] | Fn [nF] | J [nF * 7 nb] | S [nF * nF] | w [nF]
struct CorrWs {
    double *lt, *x, *xn, *F, *Fn, *J, *S, *w;
};
__host__ __device__ inline int64_t corr_ws_size(int nb, int nl) {
    const int64_t nF = 3 * (int64_t)nl + nb;
    return 6 * (int64_t)nl + 14 * (int64_t)nb + 2 * nF + nF * 7 * nb + nF * nF + nF;
}

__device__ void corr_residual(int nb, int nl, const int *links, const int *pq, const int *loc,
                              const double *q, const double *lt, const double *x, double *F) {
    for (int e = threadIdx.x; e < nl; e += blockDim.x) {
        const int n = links[e];
        const int p = pq[2 * n], qq = pq[2 * n + 1];
        const int lp = loc[p];
        double R[9];
        rotation_from_quat(x + 7 * lp + 3, R);
        const double *l = lt + 6 * e;
        double g[3];
        for (int i = 0; i < 3; ++i)
            g[i] = q[3 * (size_t)p + i] + x[7 * lp + i] +
                   (R[3 * i] * l[0] + R[3 * i + 1] * l[1] + R[3 * i + 2] * l[2]);
        if (qq >= 0) {
            const int lq = loc[qq];
            rotation_from_quat(x + 7 * lq + 3, R);
            for (int i = 0; i < 3; ++i)
                g[i] -= q[3 * (size_t)qq + i] + x[7 * lq + i] +
                        (R[3 * i] * l[3] + R[3 * i + 1] * l[4] + R[3 * i + 2] * l[5]);
        } else {
            for (int i = 0; i < 3; ++i) g[i] -= l[3 + i];
        }
        for (int i = 0; i < 3; ++i) F[3 * e + i] = g[i];
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double *d = x + 7 * b + 3;
        F[3 * nl + b] = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3] - 1.0;
    }
}

__device__ __forceinline__ void jac_block(double s, const double *p, const double *lt,
                                          double sign, double *Jrow0, int ld) {
    // rows i = 0..2 of d g / d(dq, dtheta) for one body, written at Jrow0 + i*ld
    const double pl = p[0] * lt[0] + p[1] * lt[1] + p[2] * lt[2];
    const double pxl[3] = {p[1] * lt[2] - p[2] * lt[1], p[2] * lt[0] - p[0] * lt[2],
                           p[0] * lt[1] - p[1] * lt[0]};
    for (int i = 0; i < 3; ++i) {
        double *J = Jrow0 + (size_t)i * ld;
        for (int c = 0; c < 3; ++c) J[c] += sign * (i == c ? 1.0 : 0.0);
        J[3] += sign * (2.0 * pxl[i] + 4.0 * s * lt[i]);
        for (int l = 0; l < 3; ++l) {
            // s eps_ilk lt_k: nonzero for k = 3 - i - l when i != l
            double e = 0.0;
            if (i != l) {
                const int k = 3 - i - l;
                const double sg = ((l - i + 3) % 3 == 1) ? 1.0 : -1.0;  // eps_{i,l,k}
                e = sg * lt[k];
            }
            J[4 + l] += sign * 2.0 * ((i == l ? pl : 0.0) + p[i] * lt[l] + s * e);
        }
    }
}

__global__ __launch_bounds__(256) void correct_kernel(
    const int *__restrict__ asm_body_ptr, const int *__restrict__ asm_bodies,
    const int *__restrict__ asm_link_ptr, const int *__restrict__ asm_links,
    const int *__restrict__ loc, const int *__restrict__ pq, const double *__restrict__ dl_p,
    const double *__restrict__ dl_q, const int64_t *__restrict__ ws_off, double *__restrict__ wsb,
    double *__restrict__ q, double *__restrict__ theta, double tol, int max_iter,
    int *__restrict__ iters, double *__restrict__ resid) {
    __shared__ double red[4];
    __shared__ double col[kMaxCorrRows];
    __shared__ double f_sh, fn_sh;
    __shared__ int stop_sh;
    const int a = blockIdx.x;
    const int b0 = asm_body_ptr[a], nb = asm_body_ptr[a + 1] - b0;
    const int l0 = asm_link_ptr[a], nl = asm_link_ptr[a + 1] - l0;
    const int *bodies = asm_bodies + b0;
    const int *links = asm_links + l0;
    const int nF = 3 * nl + nb, nX = 7 * nb;
    double *base = wsb + ws_off[a];
    CorrWs W;
    W.lt = base;
    W.x = W.lt + 6 * nl;
    W.xn = W.x + nX;
    W.F = W.xn + nX;
    W.Fn = W.F + nF;
    W.J = W.Fn + nF;
    W.S = W.J + (size_t)nF * nX;
    W.w = W.S + (size_t)nF * nF;
    // l~ = R(theta) dl for both link ends
    for (int e = threadIdx.x; e < nl; e += blockDim.x) {
        const int n = links[e];
        const int p = pq[2 * n], qq = pq[2 * n + 1];
        double R[9];
        rotation_from_quat(theta + 4 * (size_t)p, R);
        for (int i = 0; i < 3; ++i)
            W.lt[6 * e + i] = R[3 * i] * dl_p[3 * n] + R[3 * i + 1] * dl_p[3 * n + 1] +
                              R[3 * i + 2] * dl_p[3 * n + 2];
        if (qq >= 0) {
            rotation_from_quat(theta + 4 * (size_t)qq, R);
            for (int i = 0; i < 3; ++i)
                W.lt[6 * e + 3 + i] = R[3 * i] * dl_q[3 * n] + R[3 * i + 1] * dl_q[3 * n + 1] +
                                      R[3 * i + 2] * dl_q[3 * n + 2];
        } else {
            for (int i = 0; i < 3; ++i) W.lt[6 * e + 3 + i] = dl_q[3 * n + i];
        }
    }
    for (int k = threadIdx.x; k < nX; k += blockDim.x) W.x[k] = (k % 7 == 3) ? 1.0 : 0.0;
    __syncthreads();
    corr_residual(nb, nl, links, pq, loc, q, W.lt, W.x, W.F);
    __syncthreads();
    double acc = 0.0;
    for (int k = threadIdx.x; k < nF; k += blockDim.x) acc += W.F[k] * W.F[k];
    double f = sqrt(block_sum_c(acc, red));
    int it = 0;
    for (int outer = 0; outer < max_iter; ++outer) {
        if (!(f > tol)) break;
        // Jacobian
        for (int k = threadIdx.x; k < nF * nX; k += blockDim.x) W.J[k] = 0.0;
        __syncthreads();
        for (int e = threadIdx.x; e < nl; e += blockDim.x) {
            const int n = links[e];
            const int p = pq[2 * n], qq = pq[2 * n + 1];
            const int lp = loc[p];
            jac_block(W.x[7 * lp + 3], W.x + 7 * lp + 4, W.lt + 6 * e, 1.0,
                      W.J + (size_t)(3 * e) * nX + 7 * lp, nX);
            if (qq >= 0) {
                const int lq = loc[qq];
                jac_block(W.x[7 * lq + 3], W.x + 7 * lq + 4, W.lt + 6 * e + 3, -1.0,
                          W.J + (size_t)(3 * e) * nX + 7 * lq, nX);
            }
        }
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            for (int c = 0; c < 4; ++c) W.J[(size_t)(3 * nl + b) * nX + 7 * b + 3 + c] = 2.0 * W.x[7 * b + 3 + c];
        __syncthreads();
        double mu = f * f;
        int accepted = 0;
        for (int tries = 0; tries < 20; ++tries) {
            // S = J J^T + mu I
            for (int k = threadIdx.x; k < nF * nF; k += blockDim.x) {
                const int r = k / nF, c = k - (k / nF) * nF;
                const double *Jr = W.J + (size_t)r * nX;
                const double *Jc = W.J + (size_t)c * nX;
                double s = 0.0;
                for (int t = 0; t < nX; ++t) s += Jr[t] * Jc[t];
                W.S[k] = s + (r == c ? mu : 0.0);
            }
            for (int k = threadIdx.x; k < nF; k += blockDim.x) W.w[k] = W.F[k];
            // Cholesky (S is positive definite for mu > 0), then two triangular solves
            for (int k = 0; k < nF; ++k) {
                __syncthreads();
                if (threadIdx.x == 0) {
                    const double d = sqrt(fmax(W.S[(size_t)k * nF + k], 1e-300));
                    W.S[(size_t)k * nF + k] = d;
                    col[k] = d;
                }
                __syncthreads();
                const double inv = 1.0 / col[k];
                for (int i = k + 1 + threadIdx.x; i < nF; i += blockDim.x) {
                    const double v = W.S[(size_t)i * nF + k] * inv;
                    W.S[(size_t)i * nF + k] = v;
                    col[i] = v;
                }
                __syncthreads();
                const int wdt = nF - k - 1;
                for (int idx = threadIdx.x; idx < wdt * wdt; idx += blockDim.x) {
                    const int ii = k + 1 + idx / wdt, jj = k + 1 + (idx - (idx / wdt) * wdt);
                    if (jj <= ii) W.S[(size_t)ii * nF + jj] -= col[ii] * col[jj];
                }
            }
            for (int k = 0; k < nF; ++k) {  // L y = F
                __syncthreads();
                if (threadIdx.x == 0) W.w[k] /= W.S[(size_t)k * nF + k];
                __syncthreads();
                for (int i = k + 1 + threadIdx.x; i < nF; i += blockDim.x)
                    W.w[i] -= W.S[(size_t)i * nF + k] * W.w[k];
            }
            for (int k = nF - 1; k >= 0; --k) {  // L^T w = y
                __syncthreads();
                if (threadIdx.x == 0) W.w[k] /= W.S[(size_t)k * nF + k];
                __syncthreads();
                for (int i = threadIdx.x; i < k; i += blockDim.x)
                    W.w[i] -= W.S[(size_t)k * nF + i] * W.w[k];
            }
            __syncthreads();
            // xn = x - J^T w
            for (int c = threadIdx.x; c < nX; c += blockDim.x) {
                double s = 0.0;
                for (int r = 0; r < nF; ++r) s += W.J[(size_t)r * nX + c] * W.w[r];
                W.xn[c] = W.x[c] - s;
            }
            __syncthreads();
            corr_residual(nb, nl, links, pq, loc, q, W.lt, W.xn, W.Fn);
            __syncthreads();
            double a2 = 0.0;
            for (int k = threadIdx.x; k < nF; k += blockDim.x) a2 += W.Fn[k] * W.Fn[k];
            const double fn = sqrt(block_sum_c(a2, red));
            if (fn < f) {
                accepted = 1;
                f = fn;
                break;
            }
            mu *= 10.0;
        }
        if (!accepted) break;
        __syncthreads();
        for (int k = threadIdx.x; k < nX; k += blockDim.x) W.x[k] = W.xn[k];
        for (int k = threadIdx.x; k < nF; k += blockDim.x) W.F[k] = W.Fn[k];
        __syncthreads();
        ++it;
    }
    __syncthreads();
    // apply: q += dq, theta <- normalised(dtheta) . theta
    for (int lb = threadIdx.x; lb < nb; lb += blockDim.x) {
        const int p = bodies[lb];
        const double *X = W.x + 7 * lb;
        for (int i = 0; i < 3; ++i) q[3 * (size_t)p + i] += X[i];
        const double nrm = sqrt(X[3] * X[3] + X[4] * X[4] + X[5] * X[5] + X[6] * X[6]);
        const double a0 = X[3] / nrm, a1 = X[4] / nrm, a2 = X[5] / nrm, a3 = X[6] / nrm;
        double *t = theta + 4 * (size_t)p;
        const double c0 = t[0], c1 = t[1], c2 = t[2], c3 = t[3];
        t[0] = a0 * c0 - (a1 * c1 + a2 * c2 + a3 * c3);
        t[1] = a0 * c1 + c0 * a1 + (a2 * c3 - a3 * c2);
        t[2] = a0 * c2 + c0 * a2 + (a3 * c1 - a1 * c3);
        t[3] = a0 * c3 + c0 * a3 + (a1 * c2 - a2 * c1);
    }
    __syncthreads();
    // final link residual of the corrected state
    double g2 = 0.0;
    for (int e = threadIdx.x; e < nl; e += blockDim.x) {
        const int n = links[e];
        const int p = pq[2 * n], qq = pq[2 * n + 1];
        double R[9], v[3];
        rotation_from_quat(theta + 4 * (size_t)p, R);
        for (int i = 0; i < 3; ++i)
            v[i] = q[3 * (size_t)p + i] + R[3 * i] * dl_p[3 * n] + R[3 * i + 1] * dl_p[3 * n + 1] +
                   R[3 * i + 2] * dl_p[3 * n + 2];
        if (qq >= 0) {
            rotation_from_quat(theta + 4 * (size_t)qq, R);
            for (int i = 0; i < 3; ++i)
                v[i] -= q[3 * (size_t)qq + i] + R[3 * i] * dl_q[3 * n] +
                        R[3 * i + 1] * dl_q[3 * n + 1] + R[3 * i + 2] * dl_q[3 * n + 2];
        } else {
            for (int i = 0; i < 3; ++i) v[i] -= dl_q[3 * n + i];
        }
        g2 += v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    }
    const double g = sqrt(block_sum_c(g2, red));
    if (threadIdx.x == 0) {
        iters[a] = it;
        resid[a] = g;
    }
}

void correct_positions(hipStream_t s, const CorrectDev &C, double tol, int max_iter) {
    if (C.A <= 0) return;
    correct_kernel<<<C.A, 256, 0, s>>>(C.asm_body_ptr, C.asm_bodies, C.asm_link_ptr, C.asm_links,
                                       C.local_index, C.pq, C.dl_p, C.dl_q, C.ws_off, C.ws, C.q,
                                       C.theta, tol, max_iter, C.iters, C.resid);
}

int64_t correct_ws_doubles(int nb, int nl) { return corr_ws_size(nb, nl); }

}  // namespace arb
