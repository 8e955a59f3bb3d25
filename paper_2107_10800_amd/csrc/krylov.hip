// Dense FP64 kernels of the restarted GMRES (Sec. 3.1): Arnoldi with
// classical Gram-Schmidt applied twice, Givens rotations of the Hessenberg
// column, triangular solve and basis combination.  Reductions are two-stage
// with a fixed order, so results do not depend on scheduling.
#include "common.h"

namespace arb {

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }
constexpr int kChunk = 2048;  // elements per block in the dot-product first stage

__device__ __forceinline__ double block_sum256(double v, double *red) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) s += red[k];
    return s;
}

// partial[i * nch + chunk] = sum over the chunk of V_i . w
__global__ __launch_bounds__(256) void multidot_kernel(int64_t n, int nch,
                                                       const double *__restrict__ V, int64_t ldv,
                                                       const double *__restrict__ w,
                                                       double *__restrict__ partial) {
    __shared__ double red[4];
    const int i = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const double *v = V + (int64_t)i * ldv;
    double s = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t t = base + k;
        if (t < n) s += v[t] * w[t];
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) partial[(int64_t)i * nch + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void multidot_reduce_kernel(int nch,
                                                              const double *__restrict__ partial,
                                                              double *__restrict__ h) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int k = threadIdx.x; k < nch; k += 256) s += partial[(int64_t)i * nch + k];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) h[i] = s;
}

// w -= sum_i V_i h_i
__global__ __launch_bounds__(256) void gemv_sub_kernel(int64_t n, int k,
                                                       const double *__restrict__ V, int64_t ldv,
                                                       const double *__restrict__ h,
                                                       double *__restrict__ w) {
    __shared__ double hs[260];
    for (int i = threadIdx.x; i < k; i += 256) hs[i] = h[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += V[(int64_t)i * ldv + t] * hs[i];
    w[t] -= s;
}

__global__ __launch_bounds__(256) void gemv_set_kernel(int64_t n, int k,
                                                       const double *__restrict__ V, int64_t ldv,
                                                       const double *__restrict__ h,
                                                       double *__restrict__ out) {
    __shared__ double hs[260];
    for (int i = threadIdx.x; i < k; i += 256) hs[i] = h[i];
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += V[(int64_t)i * ldv + t] * hs[i];
    out[t] = s;
}

__global__ void scale_copy_kernel(int64_t n, const double *__restrict__ x,
                                  const double *__restrict__ alpha, double *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) y[t] = x[t] / alpha[0];
}

__global__ void axpby_kernel(int64_t n, double a, const double *__restrict__ x, double b,
                             double *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) y[t] = a * x[t] + b * y[t];
}

// h1[0..j] = first CGS pass h, h2[0..j] = second pass, hn2 = ||w||^2.
// Applies the previous rotations, builds rotation j, updates g, stores the
// rotated column in Hbar (column-major, ld = m+1), writes hn = ||w|| and the
// residual estimate |g[j+1]| to out[0], out[1].  One thread.
__device__ void arnoldi_post_dev(int j, int m, const double *h1, const double *h2, double hn2,
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

__global__ void arnoldi_post_kernel(int j, int m, const double *__restrict__ h1,
                                    const double *__restrict__ h2, const double *__restrict__ hn2,
                                    double *__restrict__ Hbar, double *__restrict__ cs,
                                    double *__restrict__ sn, double *__restrict__ g,
                                    double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    arnoldi_post_dev(j, m, h1, h2, hn2[0], Hbar, cs, sn, g, out);
}

// The whole orthogonalisation of one Arnoldi step for a system of at most
// kSmallArnoldi unknowns in one workgroup: w against V_0..V_j by classical
// Gram-Schmidt twice (w held in LDS), ||w||, then the Givens update of
// arnoldi_post.  One launch instead of nine; the same steps with a different
// summation order (one wave per dot product, lanes strided over the rows).
__global__ __launch_bounds__(1024) void arnoldi_small_kernel(
    int n, int j, int m, const double *__restrict__ V, int64_t ldv, double *__restrict__ w,
    double *__restrict__ Hbar, double *__restrict__ cs, double *__restrict__ sn,
    double *__restrict__ g, double *__restrict__ out) {
    __shared__ double ws[kSmallArnoldi];
    __shared__ double hs[2][kMaxRestart + 1];
    __shared__ double red[1024 / kWave];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    constexpr int nwave = 1024 / kWave;
    for (int t = tid; t < n; t += 1024) ws[t] = w[t];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        double *h = hs[pass];
        for (int i = wave; i <= j; i += nwave) {
            const double *v = V + (int64_t)i * ldv;
            double sacc = 0.0;
            for (int t = lane; t < n; t += kWave) sacc += v[t] * ws[t];
            for (int off = kWave / 2; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
            if (lane == 0) h[i] = sacc;
        }
        __syncthreads();
        for (int t = tid; t < n; t += 1024) {
            double acc = 0.0;
            for (int i = 0; i <= j; ++i) acc += V[(int64_t)i * ldv + t] * h[i];
            ws[t] -= acc;
        }
        __syncthreads();
    }
    double sq = 0.0;
    for (int t = tid; t < n; t += 1024) {
        sq += ws[t] * ws[t];
        w[t] = ws[t];
    }
    for (int off = kWave / 2; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (lane == 0) red[wave] = sq;
    __syncthreads();
    if (tid == 0) {
        double hn2 = 0.0;
        for (int k = 0; k < nwave; ++k) hn2 += red[k];
        arnoldi_post_dev(j, m, hs[0], hs[1], hn2, Hbar, cs, sn, g, out);
    }
}

// back substitution of the rotated (upper-triangular) Hessenberg: s = H^-1 g
__global__ void upper_solve_kernel(int k, int m, const double *__restrict__ Hbar,
                                   const double *__restrict__ g, double *__restrict__ sv) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int c = i + 1; c < k; ++c) s -= Hbar[(int64_t)c * (m + 1) + i] * sv[c];
        sv[i] = s / Hbar[(int64_t)i * (m + 1) + i];
    }
}

// b = [u_s; -F; B]
__global__ void rhs_kernel(int N, int M, int Nc, const double *__restrict__ us,
                           const double *__restrict__ F, const double *__restrict__ B,
                           double *__restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n3 = 3 * (int64_t)N, m6 = 6 * (int64_t)M;
    if (t < n3)
        b[t] = us ? us[t] : 0.0;
    else if (t < n3 + m6)
        b[t] = -F[t - n3];
    else if (t < n3 + m6 + Nc)
        b[t] = B[t - n3 - m6];
}

__global__ void g_init_kernel(int m, const double *__restrict__ beta2, double *__restrict__ g,
                              double *__restrict__ beta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double b = sqrt(beta2[0]);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = b;
    beta[0] = b;
}

void multidot(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *w,
              double *partial, double *h) {
    const int nch = (int)((n + kChunk - 1) / kChunk);
    multidot_kernel<<<dim3(nch, k), 256, 0, s>>>(n, nch, V, ldv, w, partial);
    multidot_reduce_kernel<<<k, 256, 0, s>>>(nch, partial, h);
}
void gemv_sub(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *h,
              double *w) {
    gemv_sub_kernel<<<nblk(n, 256), 256, 0, s>>>(n, k, V, ldv, h, w);
}
void gemv_set(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *h,
              double *out) {
    gemv_set_kernel<<<nblk(n, 256), 256, 0, s>>>(n, k, V, ldv, h, out);
}
void scale_copy(hipStream_t s, int64_t n, const double *x, const double *alpha_dev, double *y) {
    scale_copy_kernel<<<nblk(n, 256), 256, 0, s>>>(n, x, alpha_dev, y);
}
void axpby(hipStream_t s, int64_t n, double a, const double *x, double b, double *y) {
    axpby_kernel<<<nblk(n, 256), 256, 0, s>>>(n, a, x, b, y);
}
void arnoldi_post(hipStream_t s, int j, int m, const double *h1, const double *h2,
                  const double *hn2, double *Hbar, double *cs, double *sn, double *g,
                  double *out) {
    arnoldi_post_kernel<<<1, 64, 0, s>>>(j, m, h1, h2, hn2, Hbar, cs, sn, g, out);
}
void arnoldi_small(hipStream_t s, int64_t n, int j, int m, const double *V, int64_t ldv,
                   double *w, double *Hbar, double *cs, double *sn, double *g, double *out) {
    arnoldi_small_kernel<<<1, 1024, 0, s>>>((int)n, j, m, V, ldv, w, Hbar, cs, sn, g, out);
}
void upper_solve(hipStream_t s, int k, int m, const double *Hbar, const double *g, double *sv) {
    upper_solve_kernel<<<1, 64, 0, s>>>(k, m, Hbar, g, sv);
}
void rhs_assemble(hipStream_t s, int N, int M, int Nc, const double *us, const double *F,
                  const double *B, double *b) {
    const int64_t n = 3 * (int64_t)N + 6 * (int64_t)M + Nc;
    rhs_kernel<<<nblk(n, 256), 256, 0, s>>>(N, M, Nc, us, F, B, b);
}
void g_init(hipStream_t s, int m, const double *beta2, double *g, double *beta) {
    g_init_kernel<<<1, 64, 0, s>>>(m, beta2, g, beta);
}

}  // namespace arb
