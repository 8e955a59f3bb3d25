/*
 * Plain FP64 blob mobility sums on the CPU (Sec. 2.3, Eq. RPY): the oracle's
 * second, compiled route for u = M lambda and for the dense M, used where the
 * numpy route (rpy.py) is too slow: full products of tens of thousands of
 * blobs, oracle GMRES solves at a few tens of thousands of blobs, and the
 * timed CPU baseline.
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product path links or calls this.
 * It shares no code with the GPU library.
 *
 * Unbounded pair tensor (Rotne-Prager, Wajnryb et al.; equal radii a,
 * r = x - y, r = |r|), in units of 1/(8 pi eta):
 *   r > 2a : (1/r) [(1 + 2a^2/(3 r^2)) I + (1 - 2a^2/r^2) r r^T / r^2]
 *   r <= 2a: (4/(3a)) [(1 - 9r/(32a)) I + (3/(32 a r)) r r^T]   (r r^T term 0 at r = 0)
 * (the second is 1/(6 pi eta a) [...] times 8 pi eta).  The boundary r = 2a
 * takes the overlap branch.  Above a no-slip wall at z = 0 the image term
 * F_x F_y (G^Blake - G^Oseen)(x, y) is added, evaluated by the code
 * generated from its symbolic definition (rpy_wall_image.inc).
 *
 * Every sum runs over the sources in index order, one target per loop
 * iteration; OpenMP splits the targets over threads (no reduction across
 * threads, so the result does not depend on the thread count).
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>

#include "rpy_wall_image.inc"

/* 3x3 pair block M(x, y) in units of 1/(8 pi eta), row-major */
static void pair_block(const double *x, const double *y, double a, int wall, double M[9]) {
    const double r0 = x[0] - y[0], r1 = x[1] - y[1], r2 = x[2] - y[2];
    const double r = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    const double rv[3] = {r0, r1, r2};
    double c1, c2;
    if (r <= 2.0 * a) {
        c1 = 4.0 / (3.0 * a) * (1.0 - 9.0 * r / (32.0 * a));
        c2 = r > 0.0 ? 4.0 / (3.0 * a) * 3.0 / (32.0 * a * r) : 0.0;
    } else {
        c1 = (1.0 + 2.0 * a * a / (3.0 * r * r)) / r;
        c2 = (1.0 - 2.0 * a * a / (r * r)) / (r * r * r);
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = (i == j ? c1 : 0.0) + c2 * rv[i] * rv[j];
    if (wall) {
        double W[9];
        wall_image(x[0], x[1], x[2], y[0], y[1], y[2], a, W);
        for (int k = 0; k < 9; ++k) M[k] += W[k];
    }
}

static int set_threads(int threads) {
    if (threads > 0) omp_set_num_threads(threads);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    return used;
}

/* u[t] = sum_j M(pos[targets[t]], pos[j]) lam[j], t < nt (targets NULL: all n
 * blobs in order).  pos, lam: 3n xyz; u: 3 nt.  Returns the threads used. */
int oracle_rpy_apply(int n, const double *pos, const double *lam, double a, double eta, int wall,
                     int nt, const int *targets, double *u, int threads) {
    const int used = set_threads(threads);
    const double s = 1.0 / (8.0 * M_PI * eta);
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < nt; ++t) {
        const int i = targets ? targets[t] : t;
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, M[9];
        for (int j = 0; j < n; ++j) {
            pair_block(pos + 3 * (size_t)i, pos + 3 * (size_t)j, a, wall, M);
            const double *l = lam + 3 * (size_t)j;
            u0 += M[0] * l[0] + M[1] * l[1] + M[2] * l[2];
            u1 += M[3] * l[0] + M[4] * l[1] + M[5] * l[2];
            u2 += M[6] * l[0] + M[7] * l[1] + M[8] * l[2];
        }
        u[3 * (size_t)t] = s * u0;
        u[3 * (size_t)t + 1] = s * u1;
        u[3 * (size_t)t + 2] = s * u2;
    }
    return used;
}

/* Dense 3n x 3n mobility, row-major, xyz interleaved per blob:
 * Mout[(3i + c) 3n + 3j + d] = M(pos_i, pos_j)[c][d].  Returns the threads used. */
int oracle_rpy_matrix(int n, const double *pos, double a, double eta, int wall, double *Mout,
                      int threads) {
    const int used = set_threads(threads);
    const double s = 1.0 / (8.0 * M_PI * eta);
    const size_t ld = 3 * (size_t)n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        double M[9];
        for (int j = 0; j < n; ++j) {
            pair_block(pos + 3 * (size_t)i, pos + 3 * (size_t)j, a, wall, M);
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d)
                    Mout[(3 * (size_t)i + c) * ld + 3 * (size_t)j + d] = s * M[3 * c + d];
        }
    }
    return used;
}
