// Learned body mobility: a 7 -> 128 -> 128 -> 21 network that maps a body's
// height and orientation (plus its type) to the Cholesky factor of its scaled
// 6x6 body mobility, replacing the per-body factorisations of the block
// preconditioner of Sec. 3.1 above a wall.
//
// Arithmetic: BF16 operands on the matrix cores (v_mfma_f32_16x16x16_bf16,
// FP32 accumulation), FP32 master weights, FP32 pre-activations and bias
// gradients.  Layer l: Z = H W^T + b, H' = SiLU(Z); the output layer is linear.
// Loss: mean squared error over the 21 outputs; Adam on the FP32 weights.
//
// Layouts (row-major, padded to multiples of 16): X (B x 16, 7 used),
// H1/H2 (B x 128), Y (B x 32, 21 used); W1 (128 x 16), W2 (128 x 128),
// W3 (32 x 128) in BF16; flat FP32 parameters [W1 (128x7), b1, W2, b2,
// W3 (21x128), b3] (20,245 values).
#include "common.h"

namespace arb {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 7, kH = 128, kOut = 21, kInP = 16, kOutP = 32;
constexpr int kP = kH * kIn + kH + kH * kH + kH + kOut * kH + kOut;  // 20245
constexpr int oW1 = 0, ob1 = kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kOut * kH;

__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ __forceinline__ float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

struct GemmArgs {
    int M, N, K;
    const unsigned short *A;
    long sam, sak;
    const unsigned short *B;
    long sbk, sbn;
    int mode;            // 0: C = acc; 1: C = Z = acc + bias, Hb = bf16(silu(Z));
                         // 2: C = dZ = acc * silu'(Zs), Hb = bf16(dZ); 3: C = acc + bias
    float *C;
    long ldc;
    const float *bias;
    unsigned short *Hb;
    long ldh;
    const float *Zs;
    long ldz;
};

// one wavefront per 16 x 16 output tile, four tiles per block
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int tn = g.N / 16, tm = g.M / 16;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= tn * tm) return;  // whole wavefront exits together
    const int ti = tile / tn, tj = tile - (tile / tn) * tn;
    const long row = ti * 16 + lane % 16;
    const long col = tj * 16 + lane % 16;
    const int kq = 4 * (lane / 16);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        bf16x4 a, b;
        for (int e = 0; e < 4; ++e) {
            const long k = k0 + kq + e;
            a[e] = (short)g.A[row * g.sam + k * g.sak];
            b[e] = (short)g.B[k * g.sbk + col * g.sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    for (int e = 0; e < 4; ++e) {
        const long m = ti * 16 + kq + e, n = tj * 16 + lane % 16;
        float v = acc[e];
        if (g.mode == 0) {
            g.C[m * g.ldc + n] = v;
        } else if (g.mode == 1) {
            v += g.bias[n];
            g.C[m * g.ldc + n] = v;
            g.Hb[m * g.ldh + n] = f2bf(v * sigm(v));
        } else if (g.mode == 2) {
            const float z = g.Zs[m * g.ldz + n];
            const float s = sigm(z);
            v *= s * (1.f + z * (1.f - s));
            g.C[m * g.ldc + n] = v;
            g.Hb[m * g.ldh + n] = f2bf(v);
        } else {
            g.C[m * g.ldc + n] = v + g.bias[n];
        }
    }
}

static void gemm(hipStream_t s, const GemmArgs &g) {
    const int tiles = (g.M / 16) * (g.N / 16);
    gemm_bf16_kernel<<<(tiles + 3) / 4, 256, 0, s>>>(g);
}

// BF16 padded copies of the weights and the padded output bias
__global__ void mlp_refresh_kernel(const float *__restrict__ P, unsigned short *__restrict__ W1b,
                                   unsigned short *__restrict__ W2b,
                                   unsigned short *__restrict__ W3b, float *__restrict__ b3p) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kH * kInP) {
        const int r = t / kInP, c = t % kInP;
        W1b[t] = c < kIn ? f2bf(P[oW1 + r * kIn + c]) : 0;
    }
    if (t < kH * kH) W2b[t] = f2bf(P[oW2 + t]);
    if (t < kOutP * kH) {
        const int r = t / kH;
        W3b[t] = r < kOut ? f2bf(P[oW3 + t]) : 0;
    }
    if (t < kOutP) b3p[t] = t < kOut ? P[ob3 + t] : 0.f;
}

// X (B x 7 fp32, rows >= n zero) -> standardised BF16 padded (Bp x 16)
__global__ void mlp_pack_x_kernel(int n, int Bp, const float *__restrict__ X,
                                  const float *__restrict__ mu, const float *__restrict__ sd,
                                  unsigned short *__restrict__ Xb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * kInP) return;
    const int r = t / kInP, c = t % kInP;
    Xb[t] = (r < n && c < kIn) ? f2bf((X[r * kIn + c] - mu[c]) / sd[c]) : 0;
}

// dY = 2 (Y - T') / (n * 21), T' = (T - mu_y)/sd_y, on the first n rows / 21
// columns; loss partials
__global__ void mlp_dy_kernel(int n, int Bp, const float *__restrict__ Y,
                              const float *__restrict__ T, const float *__restrict__ mu,
                              const float *__restrict__ sd, float *__restrict__ dYf,
                              unsigned short *__restrict__ dYb, double *__restrict__ lpart) {
    __shared__ double red[4];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (t < Bp * kOutP) {
        const int r = t / kOutP, c = t % kOutP;
        float d = 0.f;
        if (r < n && c < kOut) {
            const float e = Y[t] - (T[r * kOut + c] - mu[c]) / sd[c];
            l = (double)e * e;
            d = 2.f * e / (float)(n * kOut);
        }
        dYf[t] = d;
        dYb[t] = f2bf(d);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = l;
    __syncthreads();
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// column sums of an fp32 (rows x ld) matrix over its first `rows` rows -> out[c]
__global__ void mlp_colsum_kernel(int rows, int cols, long ld, const float *__restrict__ A,
                                  float *__restrict__ out) {
    const int c = blockIdx.x;
    __shared__ float red[256];
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += 256) s += A[(long)r * ld + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && c < cols) out[c] = red[0];
}

// gather padded weight gradients into the flat layout
__global__ void mlp_gather_grad_kernel(const float *__restrict__ gW1, const float *__restrict__ gW2,
                                       const float *__restrict__ gW3, float *__restrict__ G) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kH * kIn) G[oW1 + t] = gW1[(t / kIn) * kInP + t % kIn];
    if (t < kH * kH) G[oW2 + t] = gW2[t];
    if (t < kOut * kH) G[oW3 + t] = gW3[t];
}

__global__ void mlp_adam_kernel(int n, float *__restrict__ P, const float *__restrict__ G,
                                float *__restrict__ m, float *__restrict__ v, float lr, float c1,
                                float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float g = G[t];
    const float mm = 0.9f * m[t] + 0.1f * g;
    const float vv = 0.999f * v[t] + 0.001f * g * g;
    m[t] = mm;
    v[t] = vv;
    P[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

// features of every body of the state: [z_p / a, theta (s >= 0), onehot(type)]
__global__ void mlp_features_kernel(int M, const double *__restrict__ q,
                                    const double *__restrict__ theta, const int *__restrict__ type,
                                    double a, float *__restrict__ X) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double *t = theta + 4 * (size_t)p;
    const double sg = t[0] < 0.0 ? -1.0 : 1.0;
    float *x = X + (size_t)p * kIn;
    x[0] = (float)(q[3 * (size_t)p + 2] / a);
    for (int k = 0; k < 4; ++k) x[1 + k] = (float)(sg * t[k]);
    x[5] = type[p] == 0 ? 1.f : 0.f;
    x[6] = type[p] == 1 ? 1.f : 0.f;
}

// N~_p = D^-1 L L^T D^-1 (FP64) from the network output: y = mu_y + sd_y Y,
// L_ij = y (i > j), L_ii = exp(y); flags non-finite factors
__global__ void mlp_mobility_kernel(int M, const float *__restrict__ Y, long ldy,
                                    const float *__restrict__ mu, const float *__restrict__ sd,
                                    double a, double eta, double *__restrict__ Nt,
                                    int *__restrict__ bad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    double L[36];
    for (int k = 0; k < 36; ++k) L[k] = 0.0;
    int idx = 0, ok = 1;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j) {
            const double y = (double)mu[idx] + (double)sd[idx] * (double)Y[(long)p * ldy + idx];
            ++idx;
            if (!(fabs(y) < 80.0)) ok = 0;  // also rejects NaN
            L[i * 6 + j] = (i == j) ? exp(y) : y;
        }
    if (!ok) atomicOr(bad, 1);
    const double dt = sqrt(6.0 * kPi * eta * a), dr = sqrt(8.0 * kPi * eta * a * a * a);
    double *N = Nt + 36 * (size_t)p;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += L[i * 6 + k] * L[j * 6 + k];
            N[i * 6 + j] = ok ? s / ((i < 3 ? dt : dr) * (j < 3 ? dt : dr)) : 0.0;
        }
}

// training labels: the 21 entries of chol(D N~ D) per body, log on the
// diagonal (FP64 factor, stored as float); flags bodies whose scaled mobility
// is not positive definite
__global__ void mlp_target_kernel(int M, const double *__restrict__ Nt, double a, double eta,
                                  float *__restrict__ T, int *__restrict__ bad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double dt = sqrt(6.0 * kPi * eta * a), dr = sqrt(8.0 * kPi * eta * a * a * a);
    double S[36], L[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const double v = 0.5 * (Nt[36 * (size_t)p + i * 6 + j] + Nt[36 * (size_t)p + j * 6 + i]);
            S[i * 6 + j] = v * (i < 3 ? dt : dr) * (j < 3 ? dt : dr);
            L[i * 6 + j] = 0.0;
        }
    int ok = 1;
    for (int j = 0; j < 6; ++j) {
        double d = S[j * 6 + j];
        for (int k = 0; k < j; ++k) d -= L[j * 6 + k] * L[j * 6 + k];
        if (!(d > 0.0)) {
            ok = 0;
            d = 1e-300;
        }
        L[j * 6 + j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double v = S[i * 6 + j];
            for (int k = 0; k < j; ++k) v -= L[i * 6 + k] * L[j * 6 + k];
            L[i * 6 + j] = v / L[j * 6 + j];
        }
    }
    if (!ok) atomicOr(bad, 1);
    int idx = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j <= i; ++j)
            T[(size_t)p * kOut + idx++] = (float)(i == j ? log(L[i * 6 + j]) : L[i * 6 + j]);
}

void mlp_targets(hipStream_t s, int M, const double *Nt, double a, double eta, float *T, int *bad) {
    if (M > 0) mlp_target_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, Nt, a, eta, T, bad);
}

// ---------------------------------------------------------------- host side
struct MlpBuffers {
    float *P, *m, *v, *G;
    unsigned short *W1b, *W2b, *W3b;
    float *b3p;
    float *in_mu, *in_sd, *out_mu, *out_sd;  // 16, 16, 32, 32
    // batch workspace (Bp rows)
    unsigned short *Xb, *H1b, *H2b, *dYb, *dZ2b, *dZ1b;
    float *Z1, *Z2, *Y, *dYf, *dZ2f, *dZ1f, *gW1, *gW2, *gW3;
    double *lpart;
};

int64_t mlp_workspace_bytes(int Bp) {
    const int64_t b = Bp;
    return 2 * (b * kInP + 2 * b * kH + b * kOutP + 2 * b * kH) +
           4 * (2 * b * kH + 2 * b * kOutP + 2 * b * kH + kH * kInP + kH * kH + kOutP * kH) +
           8 * ((b * kOutP + 255) / 256 + 16) + 4096;
}

static MlpBuffers carve(void *params, void *ws, int Bp) {
    MlpBuffers B;
    char *p = (char *)params;
    B.P = (float *)p;
    B.m = B.P + kP;
    B.v = B.m + kP;
    B.G = B.v + kP;
    B.b3p = B.G + kP;
    B.W1b = (unsigned short *)(B.b3p + kOutP);
    B.W2b = B.W1b + kH * kInP;
    B.W3b = B.W2b + kH * kH;
    B.in_mu = (float *)(B.W3b + kOutP * kH);
    B.in_sd = B.in_mu + kInP;
    B.out_mu = B.in_sd + kInP;
    B.out_sd = B.out_mu + kOutP;
    char *w = (char *)ws;
    auto take = [&](size_t bytes) {
        char *r = w;
        w += (bytes + 255) & ~(size_t)255;
        return r;
    };
    const size_t b = Bp;
    B.Xb = (unsigned short *)take(2 * b * kInP);
    B.H1b = (unsigned short *)take(2 * b * kH);
    B.H2b = (unsigned short *)take(2 * b * kH);
    B.dYb = (unsigned short *)take(2 * b * kOutP);
    B.dZ2b = (unsigned short *)take(2 * b * kH);
    B.dZ1b = (unsigned short *)take(2 * b * kH);
    B.Z1 = (float *)take(4 * b * kH);
    B.Z2 = (float *)take(4 * b * kH);
    B.Y = (float *)take(4 * b * kOutP);
    B.dYf = (float *)take(4 * b * kOutP);
    B.dZ2f = (float *)take(4 * b * kH);
    B.dZ1f = (float *)take(4 * b * kH);
    B.gW1 = (float *)take(4 * kH * kInP);
    B.gW2 = (float *)take(4 * kH * kH);
    B.gW3 = (float *)take(4 * kOutP * kH);
    B.lpart = (double *)take(8 * ((b * kOutP + 255) / 256 + 16));
    return B;
}

int64_t mlp_param_bytes() {
    return (int64_t)4 * (4 * kP + kOutP) + 2 * (kH * kInP + kH * kH + kOutP * kH) +
           4 * (2 * kInP + 2 * kOutP) + 256;
}
// bytes of the parameter block that set_params clears (weights, Adam state, gradient)
int64_t mlp_state_bytes() { return (int64_t)4 * 4 * kP; }

// standardisation constants (host arrays: 7, 7, 21, 21); sd must be > 0
void mlp_set_scaling(hipStream_t s, void *params, const float *in_mu, const float *in_sd,
                     const float *out_mu, const float *out_sd) {
    MlpBuffers B = carve(params, params, 16);
    float h[2 * kInP + 2 * kOutP];
    for (int k = 0; k < kInP; ++k) {
        h[k] = k < kIn ? in_mu[k] : 0.f;
        h[kInP + k] = k < kIn ? in_sd[k] : 1.f;
    }
    for (int k = 0; k < kOutP; ++k) {
        h[2 * kInP + k] = k < kOut ? out_mu[k] : 0.f;
        h[2 * kInP + kOutP + k] = k < kOut ? out_sd[k] : 1.f;
    }
    (void)hipMemcpyAsync(B.in_mu, h, sizeof(h), hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
}
int mlp_n_params() { return kP; }

void mlp_refresh(hipStream_t s, void *params) {
    MlpBuffers B = carve(params, params, 16);
    mlp_refresh_kernel<<<(kH * kH + 255) / 256, 256, 0, s>>>(B.P, B.W1b, B.W2b, B.W3b, B.b3p);
}

// forward of n rows (Bp = n rounded up to 16): returns Y (Bp x 32 fp32) in ws
float *mlp_forward(hipStream_t s, void *params, void *ws, int n, int Bp, const float *X) {
    MlpBuffers B = carve(params, ws, Bp);
    mlp_pack_x_kernel<<<(Bp * kInP + 255) / 256, 256, 0, s>>>(n, Bp, X, B.in_mu, B.in_sd, B.Xb);
    GemmArgs g{};
    g = GemmArgs{Bp, kH, kInP, B.Xb, kInP, 1, B.W1b, 1, kInP, 1, B.Z1, kH, B.P + ob1, B.H1b, kH,
                 nullptr, 0};
    gemm(s, g);
    g = GemmArgs{Bp, kH, kH, B.H1b, kH, 1, B.W2b, 1, kH, 1, B.Z2, kH, B.P + ob2, B.H2b, kH,
                 nullptr, 0};
    gemm(s, g);
    g = GemmArgs{Bp, kOutP, kH, B.H2b, kH, 1, B.W3b, 1, kH, 3, B.Y, kOutP, B.b3p, nullptr, 0,
                 nullptr, 0};
    gemm(s, g);
    return B.Y;
}

// forward + backward of n rows; gradient into the flat G (params buffer),
// loss partial sums in lpart (returns the count of partials)
int mlp_backward(hipStream_t s, void *params, void *ws, int n, int Bp, const float *X,
                 const float *T, double **lpart) {
    mlp_forward(s, params, ws, n, Bp, X);
    MlpBuffers B = carve(params, ws, Bp);
    const int nlp = (Bp * kOutP + 255) / 256;
    mlp_dy_kernel<<<nlp, 256, 0, s>>>(n, Bp, B.Y, T, B.out_mu, B.out_sd, B.dYf, B.dYb, B.lpart);
    GemmArgs g{};
    // dW3 = dY^T H2 (32 x 128)
    g = GemmArgs{kOutP, kH, Bp, B.dYb, 1, kOutP, B.H2b, kH, 1, 0, B.gW3, kH, nullptr, nullptr, 0,
                 nullptr, 0};
    gemm(s, g);
    mlp_colsum_kernel<<<kOutP, 256, 0, s>>>(Bp, kOut, kOutP, B.dYf, B.G + ob3);
    // dZ2 = (dY W3) * silu'(Z2)
    g = GemmArgs{Bp, kH, kOutP, B.dYb, kOutP, 1, B.W3b, kH, 1, 2, B.dZ2f, kH, nullptr, B.dZ2b, kH,
                 B.Z2, kH};
    gemm(s, g);
    // dW2 = dZ2^T H1
    g = GemmArgs{kH, kH, Bp, B.dZ2b, 1, kH, B.H1b, kH, 1, 0, B.gW2, kH, nullptr, nullptr, 0,
                 nullptr, 0};
    gemm(s, g);
    mlp_colsum_kernel<<<kH, 256, 0, s>>>(Bp, kH, kH, B.dZ2f, B.G + ob2);
    // dZ1 = (dZ2 W2) * silu'(Z1)
    g = GemmArgs{Bp, kH, kH, B.dZ2b, kH, 1, B.W2b, kH, 1, 2, B.dZ1f, kH, nullptr, B.dZ1b, kH,
                 B.Z1, kH};
    gemm(s, g);
    // dW1 = dZ1^T X (128 x 16)
    g = GemmArgs{kH, kInP, Bp, B.dZ1b, 1, kH, B.Xb, kInP, 1, 0, B.gW1, kInP, nullptr, nullptr, 0,
                 nullptr, 0};
    gemm(s, g);
    mlp_colsum_kernel<<<kH, 256, 0, s>>>(Bp, kH, kH, B.dZ1f, B.G + ob1);
    mlp_gather_grad_kernel<<<(kH * kH + 255) / 256, 256, 0, s>>>(B.gW1, B.gW2, B.gW3, B.G);
    *lpart = B.lpart;
    return nlp;
}

void mlp_adam(hipStream_t s, void *params, float lr, int t) {
    MlpBuffers B = carve(params, params, 16);
    const float c1 = 1.f - powf(0.9f, (float)t), c2 = 1.f - powf(0.999f, (float)t);
    mlp_adam_kernel<<<(kP + 255) / 256, 256, 0, s>>>(kP, B.P, B.G, B.m, B.v, lr, c1, c2);
    mlp_refresh(s, params);
}

void mlp_features(hipStream_t s, int M, const double *q, const double *theta, const int *type,
                  double a, float *X) {
    if (M > 0) mlp_features_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, q, theta, type, a, X);
}

void mlp_mobility(hipStream_t s, void *params, int M, const float *Y, double a, double eta,
                  double *Nt, int *bad) {
    MlpBuffers B = carve(params, params, 16);
    if (M > 0)
        mlp_mobility_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, Y, kOutP, B.out_mu, B.out_sd, a, eta,
                                                            Nt, bad);
}

// destandardised outputs y = mu_y + sd_y Y (Bp x 32 in place -> host copy by caller)
__global__ void mlp_destd_kernel(int n, float *__restrict__ Y, const float *__restrict__ mu,
                                 const float *__restrict__ sd) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kOutP) return;
    const int c = t % kOutP;
    Y[t] = mu[c] + sd[c] * Y[t];
}
void mlp_destandardize(hipStream_t s, void *params, int n, float *Y) {
    MlpBuffers B = carve(params, params, 16);
    if (n > 0) mlp_destd_kernel<<<(n * kOutP + 255) / 256, 256, 0, s>>>(n, Y, B.out_mu, B.out_sd);
}

}  // namespace arb
