// Reconstruction of articulated bodies from their orientations (Sec. 4.1,
// Eq. Pq_eq_z, Eq. pseudo-inv-sol, Eq. reconst-up-COM) and the link residual
// g_n = q_p + R(theta_p) dl_np - q_q - R(theta_q) dl_nq (Eq. constraint).
//
// For one articulated body a with M_a bodies and P_a links the link equations
// at fixed orientations read (Phat (x) I3) q = -z, Phat the P_a x M_a
// incidence matrix (+1 at the + body of a link, -1 at the - body) and
// z_n = R_p dl_np - R_q dl_nq.  For a connected body graph the pseudo-inverse
// is Phat^+ = (L + 1 1^T / M_a)^-1 Phat^T with L = Phat^T Phat the graph
// Laplacian (the all-ones vector spans its null space and Phat 1 = 0), so
//     q~ = -G b,  G = (L + 1 1^T / M_a)^-1 (precomputed),  b = Phat^T z,
// and q~ has zero mean.  The bodies are placed at q~ + q_COM, q_COM the mean
// of the incoming tracking points.  A link to a fixed lab point (- body = -1)
// contributes +1 on the diagonal of L and z_n = R_p dl_np - (that point); an
// articulated body with such a link has no null space: G = L^-1, no COM term.
//
// One workgroup per articulated body.  Every loop is bounded by the sizes of
// the body; every thread follows the same barriers.
#include "common.h"

namespace arb {

namespace {

__device__ __forceinline__ void rot_apply(const double *R, const double *v, double *o) {
    o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}

constexpr int kReconThreads = 256;

// block-wide sum (op 0) or max (op 1); the result reaches every thread
template <int OP>
__device__ double block_reduce(double v, double *red) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = OP == 0 ? v + o : fmax(v, o);
    }
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < kReconThreads / kWave; ++k) r = OP == 0 ? r + red[k] : fmax(r, red[k]);
    return r;
}

// g_n of link n with the current positions and orientations
__device__ __forceinline__ void link_g(const ReconDev &D, int n, double *g) {
    const int p = D.pq[2 * n], qq = D.pq[2 * n + 1];
    double R[9], v[3];
    rotation_from_quat(D.theta + 4 * (size_t)p, R);
    rot_apply(R, D.dl_p + 3 * (size_t)n, v);
    for (int i = 0; i < 3; ++i) g[i] = D.q[3 * (size_t)p + i] + v[i];
    if (qq >= 0) {
        rotation_from_quat(D.theta + 4 * (size_t)qq, R);
        rot_apply(R, D.dl_q + 3 * (size_t)n, v);
        for (int i = 0; i < 3; ++i) g[i] -= D.q[3 * (size_t)qq + i] + v[i];
    } else {
        for (int i = 0; i < 3; ++i) g[i] -= D.dl_q[3 * (size_t)n + i];
    }
}

__global__ __launch_bounds__(kReconThreads) void reconstruct_kernel(ReconDev D, int rebuild) {
    __shared__ double red[kReconThreads / kWave];
    const int a = blockIdx.x;
    const int tid = threadIdx.x;
    const int b0 = D.asm_body_ptr[a], nb = D.asm_body_ptr[a + 1] - b0;
    const int l0 = D.asm_link_ptr[a], nl = D.asm_link_ptr[a + 1] - l0;
    if (rebuild) {
        const bool anch = D.anchored[a] != 0;
        // centre of the incoming tracking points
        double c[3] = {0.0, 0.0, 0.0};
        if (!anch) {
            double s[3] = {0.0, 0.0, 0.0};
            for (int k = tid; k < nb; k += kReconThreads) {
                const int p = D.asm_bodies[b0 + k];
                for (int i = 0; i < 3; ++i) s[i] += D.q[3 * (size_t)p + i];
            }
            for (int i = 0; i < 3; ++i) c[i] = block_reduce<0>(s[i], red) / nb;
        }
        // z_n = R_p dl_np - R_q dl_nq
        for (int e = tid; e < nl; e += kReconThreads) {
            const int n = D.asm_links[l0 + e];
            const int p = D.pq[2 * n], qq = D.pq[2 * n + 1];
            double R[9], v[3], z[3];
            rotation_from_quat(D.theta + 4 * (size_t)p, R);
            rot_apply(R, D.dl_p + 3 * (size_t)n, z);
            if (qq >= 0) {
                rotation_from_quat(D.theta + 4 * (size_t)qq, R);
                rot_apply(R, D.dl_q + 3 * (size_t)n, v);
            } else {
                for (int i = 0; i < 3; ++i) v[i] = D.dl_q[3 * (size_t)n + i];
            }
            for (int i = 0; i < 3; ++i) D.z[3 * (size_t)(l0 + e) + i] = z[i] - v[i];
        }
        __syncthreads();
        // b = Phat^T z: each body sums its links with their signs
        for (int k = tid; k < nb; k += kReconThreads) {
            double s[3] = {0.0, 0.0, 0.0};
            for (int j = D.adj_ptr[b0 + k]; j < D.adj_ptr[b0 + k + 1]; ++j) {
                const int e2 = D.adj[j];
                const double sg = (e2 & 1) ? -1.0 : 1.0;
                const double *z = D.z + 3 * (size_t)(l0 + (e2 >> 1));
                for (int i = 0; i < 3; ++i) s[i] += sg * z[i];
            }
            for (int i = 0; i < 3; ++i) D.b[3 * (size_t)(b0 + k) + i] = s[i];
        }
        __syncthreads();
        // q = -G b + q_COM
        const double *G = D.G + D.g_off[a];
        for (int k = tid; k < nb; k += kReconThreads) {
            double s[3] = {0.0, 0.0, 0.0};
            const double *Gk = G + (size_t)k * nb;
            for (int j = 0; j < nb; ++j) {
                const double gkj = Gk[j];
                const double *bj = D.b + 3 * (size_t)(b0 + j);
                for (int i = 0; i < 3; ++i) s[i] = fma(gkj, bj[i], s[i]);
            }
            const int p = D.asm_bodies[b0 + k];
            for (int i = 0; i < 3; ++i) D.q[3 * (size_t)p + i] = c[i] - s[i];
        }
        __syncthreads();
    }
    // residual of every link of the articulated body
    double gi = 0.0, g2 = 0.0;
    for (int e = tid; e < nl; e += kReconThreads) {
        double g[3];
        link_g(D, D.asm_links[l0 + e], g);
        for (int i = 0; i < 3; ++i) {
            gi = fmax(gi, fabs(g[i]));
            g2 = fma(g[i], g[i], g2);
        }
    }
    gi = block_reduce<1>(gi, red);
    g2 = block_reduce<0>(g2, red);
    if (tid == 0) {
        D.ginf[a] = gi;
        D.g2[a] = g2;
    }
}

}  // namespace

void reconstruct(hipStream_t s, const ReconDev &D, int rebuild) {
    if (D.A > 0) reconstruct_kernel<<<D.A, kReconThreads, 0, s>>>(D, rebuild);
}

}  // namespace arb
