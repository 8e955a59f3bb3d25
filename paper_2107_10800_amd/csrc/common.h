// Internal declarations shared by the HIP translation units of libarb.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "arb.h"

namespace arb {

constexpr int kTile = 256;          // sources per LDS tile == threads per pair block
constexpr int kWave = 64;           // CDNA wavefront
constexpr double kPi = 3.14159265358979323846;

// R(theta) = 2 [p p^T + s p^x + (s^2 - 1/2) I] of a quaternion theta = (s, p),
// row-major (App. B, Eq. rot_mat): a rotation for unit theta; the position
// correction also evaluates it at its non-unit iterates, as App. B writes it
__device__ __forceinline__ void rotation_from_quat(const double *t, double *R) {
    const double s = t[0], p0 = t[1], p1 = t[2], p2 = t[3];
    const double d = s * s - 0.5;
    R[0] = 2.0 * (p0 * p0 + d);
    R[1] = 2.0 * (p0 * p1 - s * p2);
    R[2] = 2.0 * (p0 * p2 + s * p1);
    R[3] = 2.0 * (p1 * p0 + s * p2);
    R[4] = 2.0 * (p1 * p1 + d);
    R[5] = 2.0 * (p1 * p2 - s * p0);
    R[6] = 2.0 * (p2 * p0 - s * p1);
    R[7] = 2.0 * (p2 * p1 + s * p0);
    R[8] = 2.0 * (p2 * p2 + d);
}

// ---------------------------------------------------------------- device buffer
// bumped whenever any device buffer is (re)allocated: captured HIP graphs that
// hold buffer addresses are rebuilt after it changes
inline std::atomic<unsigned long long> &alloc_generation() {
    static std::atomic<unsigned long long> g{0};
    return g;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow-only; contents are not preserved when growing
    hipError_t ensure(size_t nbytes) {
        if (nbytes <= bytes && p) return hipSuccess;
        release();
        size_t nb = nbytes ? nbytes : 16;
        hipError_t e = hipMalloc(&p, nb);
        if (e == hipSuccess) bytes = nb;
        ++alloc_generation();
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------- fast product (fmm.hip)
constexpr int kFmmMaxOrder = 8;                                          // Chebyshev points per direction
constexpr int kFmmMaxP = kFmmMaxOrder * kFmmMaxOrder * kFmmMaxOrder;   // proxies per cell
constexpr int kFmmMaxLevel = 16;
constexpr int kFmmDefaultOrder = 6;

// octree and proxy buffers of the fast product; cells of all levels 0..L in
// Morton order, level l at [lvl[l], lvl[l+1])
struct FmmHostCache;  // host buffers of the tree build, kept between builds (fmm.hip)
struct FmmState {
    std::shared_ptr<FmmHostCache> host;
    DevBuf perm, cc, rng, parent, kids, il_ptr, il, near_ptr, nearl, work, tab, shi, slo, slam,
        qhat, v, slam2, qhat2, v2;  // second channel: the torques of single-blob bodies
    DevBuf vsplit;  // M2L sums of the parts of split interaction lists (splits > 1)
    int N = 0, L = 0, n = 0, P = 0, ncell = 0, nleaf = 0, nwork = 0, channels = 1;
    int splits = 1;  // M2L work items per cell
    int64_t n_il = 0, n_near_pairs = 0;  // interaction-list entries, direct pairs
    int64_t n_m2l_pairs = 0;             // M2L pair evaluations per product
    std::vector<int> lvl;
    double o[3] = {0.0, 0.0, 0.0}, S = 0.0;  // root cube in units of a
    long long version = 0;                   // bumped by every build
    double build_ms = 0.0;                   // host time of the last build
    bool ready = false, dirty = true;
};
// tree of N blobs (positions in units of length on the device, hi/lo as
// prep_positions makes them); order = Chebyshev points per direction (0: the
// default), levels = leaf level (0: chosen, from leaf, the mean blobs per leaf
// aimed at, or when leaf = 0 the level with the fewest pair evaluations);
// channels = 2 adds the torque channel of single-blob bodies.  Returns 0 or an
// ARB_E_* code with *msg set.
int fmm_build(FmmState &F, hipStream_t s, int N, const double *pos_dev, const float4 *hi,
              const float4 *lo, double a, int order, int levels, int leaf, int channels,
              std::string *msg);
// partial[c][i] (3 x N, original order) = the approximation of M_{a=1} lambda,
// M in units of 1/(8 pi eta) with positions in units of a; fp64: lambda and
// every sum in double (linear in lambda to double rounding), else in float
void fmm_apply(const FmmState &F, hipStream_t s, bool wall, bool fp64, const double *lam,
               double *partial);
// single-blob bodies (unbounded, generalised RPY, a tree built with channels = 2):
// partial[j][i] (6 x M, original order) = the approximation of N_{a=1} (f, tau / a)
// with positions in units of a; the caller scales u by 1/(8 pi eta a), w by
// 1/(8 pi eta a^2)
void fmm_apply6(const FmmState &F, hipStream_t s, bool fp64, const double *x6, double inv_a,
                double *partial);

// ---------------------------------------------------------------- kernel entry points
// Pair sum u_i = sum_j M_ij lambda_j (Sec. 2.3): partial sums per source slice,
// then an ordered reduction.  Positions are prepared by prep_positions().
// box (may be null): 2 float4 per 64-blob tile, its bounding box and largest
// |coordinate| (pair_sym's far test)
// perm (may be null): entry i of the outputs holds blob perm[i]
// (sx, sy) is subtracted from every position (the products do not depend on a
// shift parallel to the wall; a centred domain keeps |x| and the FP32 rounding
// of the split positions small)
void prep_positions(hipStream_t s, int N, const double *pos_aos, double a, double4 *p64,
                    float4 *hi, float4 *lo, float4 *box, const int *perm, double sx = 0.0,
                    double sy = 0.0);
// device address of the allocation-free entry point's scratch array for the
// current device (noalloc.hip), looked up once per device; 0 when known
int noalloc_setup(int device);
// source slices of the target-parallel kernel when none are given: doubled while
// the grid stays within about 2,048 workgroups and every slice keeps a tile
int heuristic_slices(int N);
// returns the number of slices written (clamped to the tile count)
// small systems: target-parallel sums over runs of kSmallRun sources, one 64-lane
// workgroup per (64 targets, run); partial holds ceil(N / kSmallRun) slices;
// returns that count
constexpr int kSmallPairN = 1024;
constexpr int kSmallRun = 16;
int pair_partial_small(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
                       const float4 *hi, const float4 *lo, const double *lam, const int *perm,
                       double a, double *partial);
// positions in the order of perm (may be null), lambda in blob order, partial in
// the positions' order
int pair_partial(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
                  const float4 *hi, const float4 *lo, const double *lam, const int *perm,
                  double a, int slices, double *partial);
// out_i = scale * sum_s partial[s][c][i]  -  (K U)_i   (the K term only if U != nullptr)
void pair_reduce(hipStream_t s, int N, int slices, const double *partial, double scale,
                 double *out, const double *U, const int *body_of_blob, const double *dvec,
                 const int *perm);
int pair_wall_violation(hipStream_t s, int N, const double4 *p64, double a, int *flag_dev,
                        int *flag_host);
// symmetric pair sums, FP32 (hi/lo) or FP64 (p64) (pair_sym.hip): u [3][N]
// unscaled, accumulated into u (cleared first by pair_sym_clear)
void pair_sym_clear(hipStream_t s, int N, double *u);
void pair_sym(hipStream_t s, int precision, bool wall, int N, const double4 *p64,
              const float4 *hi, const float4 *lo, const float4 *box, const double *lam,
              const int *perm, double a, const int4 *work, int n_work, double *u);
std::vector<int4> pair_sym_worklist(int N, int R);

// Rigid-body kinematics (Sec. 2.1, 2.3, App. B)
void rotations(hipStream_t s, int M, const double *theta, double *R9);
void blob_geometry(hipStream_t s, int N, const int *body_of_blob, const double *q,
                   const double *R9, const double *r_ref, double *pos_aos, double *dvec);
void K_apply(hipStream_t s, int N, const int *body_of_blob, const double *dvec,
             const double *U, double *out);
// out_p = sign * (K^T lambda)_p + (C^T phi)_p  (phi may be null)
void KT_CT_apply(hipStream_t s, int M, const int *blob_off, const double *dvec,
                 const double *lam, double sign, const int *brow_ptr, const int *brow_ent,
                 const double *crow, const double *phi, double *out);
void constraint_rows(hipStream_t s, int Nc, const int *row_p, const int *row_q,
                     const int *row_kind, const int *row_src, const int *row_m,
                     const double *R9, const double *dl_p, const double *dl_q,
                     const double *dldot_p, const double *dldot_q, const double *proj,
                     const double *gcoef, const double *grhs, double *crow, double *B);
void C_apply(hipStream_t s, int Nc, const int *row_p, const int *row_q, const double *crow,
             const double *U, double *out);
void euler_update(hipStream_t s, int M, const double *U, double dt, double *q, double *theta);

// Block-diagonal preconditioner (Sec. 3.1)
struct PrecondDev {
    int M = 0, A = 0;
    const int *blob_off = nullptr;     // M+1
    const int64_t *mat_off = nullptr;  // M+1, doubles
    const int64_t *z_off = nullptr;    // M+1, doubles (18 n_p per body)
    const int *asm_body_ptr = nullptr, *asm_bodies = nullptr;
    const int *asm_row_ptr = nullptr, *asm_rows = nullptr;
    const int64_t *asm_mat_off = nullptr;
    const int *row_p = nullptr, *row_q = nullptr;
    const int *brow_ptr = nullptr, *brow_ent = nullptr;
    const double *crow = nullptr;
    double *mats = nullptr;   // per-body M_pp, Cholesky in place
    double *minv = nullptr;   // per-body M_pp^-1 (same offsets as mats)
    double *ldiag = nullptr;  // diag(L) per body (3N)
    double *dinv = nullptr;   // inverses of L's 32 x 32 diagonal blocks per body
    double *Z = nullptr;      // per-body Z_p = M_pp^-1 K_p (3n_p x 6)
    double *Nt = nullptr;     // per-body N~_p (36)
    double *G = nullptr;      // per-assembly G~_a
    double *S = nullptr;      // per-assembly scratch (S_a and its factor)
    int asm_max_rows = 0;     // largest assembly (constraint rows)
    double *asm_dinv = nullptr;  // diagonal-block inverses of the assemblies' factors
    int *asm_fail = nullptr;     // per assembly: 1 if S_a failed the pivot test
    int *body_pinv = nullptr;    // per body: 1 if R_p = K^T M^-1 K awaits the pseudo-inverse
    int *status = nullptr;    // [0] not-SPD body+1, [1] G~ pinv count, [2] below wall,
                              // [3] N~ with dropped eigenvalues
    double *tmp = nullptr;    // apply scratch: U-hat (6M)
    // learned variant: per-type body-frame blocks rotated by R_p
    int learned = 0;
    const int *type = nullptr;
    const int64_t *tmat_off = nullptr, *tz_off = nullptr;
    const double *tminv = nullptr, *tZ = nullptr, *R9 = nullptr;
    const double *lcorr = nullptr;  // learned: per body N~_f, E1, E2 (108); null: body frame
    double *stmp = nullptr;         // learned apply scratch: s = Z_f^T r_lam (6M)
};
void precond_assemble(hipStream_t s, const PrecondDev &P, const double *pos_aos, double a,
                      double eta, bool wall);

// A small multiblob system for gmres_small_cycle (small.hip): the state's arrays
// (positions in the pair kernels' order, perm may be null), the exact block
// preconditioner, FP64 pair sums.  tpt threads share a target (a power of 2 <= 64);
// assemblies have at most 64 rows.
struct SmallSystem {
    int N = 0, M = 0, Nc = 0, A = 0, tpt = 1;
    int64_t n = 0;
    // sizes of the arrays staged in LDS: M_pp^-1 and Z_p of all bodies, G~ of all
    // assemblies (doubles), the bodies' row entries
    int64_t n_minv = 0, n_z = 0, n_g = 0;
    int n_brow_ent = 0;
    bool wall = false;
    double a = 1.0, scale = 0.0;  // blob radius, 1 / (8 pi eta)
    const double4 *p64 = nullptr;
    const int *perm = nullptr, *bob = nullptr, *blob_off = nullptr;
    const double *dvec = nullptr;
    const int *brow_ptr = nullptr, *brow_ent = nullptr, *row_p = nullptr, *row_q = nullptr;
    const double *crow = nullptr;
    const int64_t *mat_off = nullptr, *z_off = nullptr;
    const double *minv = nullptr, *Z = nullptr, *Nt = nullptr;
    const int *asm_row_ptr = nullptr, *asm_rows = nullptr;
    const int64_t *asm_mat_off = nullptr;
    const double *G = nullptr;
};
// where gmres_small_cycle keeps everything in LDS, in units of 8 bytes for the
// doubles (and 64-bit offsets) and of 4 bytes for the ints after them
struct SmallLayout {
    size_t vs, zs, ws, us, w6, yv, p64, dvec, minv, Z, Nt, G, crow, mat_off, z_off, asm_mat_off,
        ints;
    size_t bob, blob_off, brow_ptr, brow_ent, row_p, row_q, asm_row_ptr, asm_rows, slot_a, perm,
        n_ints;
    size_t bytes;
};
__host__ __device__ inline SmallLayout small_layout(const SmallSystem &S) {
    SmallLayout L;
    size_t o = 0;
    auto d = [&](size_t cnt) {
        const size_t at = (o + 1) & ~(size_t)1;  // 16-byte aligned
        o = at + cnt;
        return at;
    };
    L.vs = d(S.n);
    L.zs = d(S.n);
    L.ws = d(S.n);
    L.us = d(6 * (size_t)S.M);
    L.w6 = d(6 * (size_t)S.M);
    L.yv = d(S.Nc);
    L.p64 = d(4 * (size_t)S.N);
    L.dvec = d(3 * (size_t)S.N);
    L.minv = d(S.n_minv);
    L.Z = d(S.n_z);
    L.Nt = d(36 * (size_t)S.M);
    L.G = d(S.n_g);
    L.crow = d(12 * (size_t)S.Nc);
    L.mat_off = d(S.M + 1);
    L.z_off = d(S.M + 1);
    L.asm_mat_off = d(S.A + 1);
    L.ints = o;
    size_t q = 0;
    L.bob = q;
    q += S.N;
    L.blob_off = q;
    q += S.M + 1;
    L.brow_ptr = q;
    q += S.M + 1;
    L.brow_ent = q;
    q += S.n_brow_ent;
    L.row_p = q;
    q += S.Nc;
    L.row_q = q;
    q += S.Nc;
    L.asm_row_ptr = q;
    q += S.A + 1;
    L.asm_rows = q;
    q += S.Nc;
    L.slot_a = q;
    q += S.Nc;
    L.perm = q;
    q += S.perm ? S.N : 0;
    L.n_ints = q;
    L.bytes = 8 * L.ints + 4 * L.n_ints;
    return L;
}
constexpr size_t kSmallCycleLds = 144 * 1024;  // arena limit (bytes)
constexpr int kSmallCycleN = 128;      // blobs
constexpr int kSmallCycleRows = 64;    // rows of the largest assembly
// Arnoldi steps 0 .. budget-1 of one cycle from v_0 = V[0..n) (Hbar, cs, sn, g as
// the per-step path leaves them); steps[2 j] = h_{j+1,j}, steps[2 j + 1] = the
// residual estimate, steps[2 m] = the steps taken (the cycle ends early when the
// estimate reaches target or h_{j+1,j} = 0)
hipError_t gmres_small_cycle(hipStream_t s, const SmallSystem &S, int m, int budget,
                             double target, double *V, double *Hbar, double *cs, double *sn,
                             double *g, double *steps);
// max_m = largest 3 n_p of the batch
hipError_t precond_factor(hipStream_t s, const PrecondDev &P, const double *dvec, int max_m);
// whether precond_factor leaves the Cholesky factors in P.mats (else the blocks
// themselves: the inverse is formed out of place)
bool precond_factor_in_place(int max_m);
int64_t precond_dinv_size(int64_t n_blobs, int M);
hipError_t precond_assembly(hipStream_t s, const PrecondDev &P);
void precond_apply(hipStream_t s, const PrecondDev &P, int N, const double *r, double *z);
void rotate_body_mobility(hipStream_t s, int M, const int *type, const double *tNt,
                          const double *R9, double *Nt);
void learned_correction(hipStream_t s, int M, const int *type, const double *tNt,
                        const double *R9, const double *Nw, double *out, int *bad);

// Dense helpers for the Krylov solver (FP64, Sec. 3.1)
void multidot(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *w,
              double *partial, double *h);
void gemv_sub(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *h,
              double *w);
void gemv_set(hipStream_t s, int64_t n, int k, const double *V, int64_t ldv, const double *h,
              double *out);
void scale_copy(hipStream_t s, int64_t n, const double *x, const double *alpha_dev, double *y);
void axpby(hipStream_t s, int64_t n, double a, const double *x, double b, double *y);
// largest system (unknowns) whose Arnoldi orthogonalisation runs in one
// workgroup (arnoldi_small), and the largest restart length
constexpr int kSmallArnoldi = 4096;
constexpr int kMaxRestart = 256;
// CGS2 + norm + Givens update of Arnoldi step j for n <= kSmallArnoldi in one
// launch: w is orthogonalised in place; out[0] = ||w||, out[1] = |g[j+1]|
void arnoldi_small(hipStream_t s, int64_t n, int j, int m, const double *V, int64_t ldv,
                   double *w, double *Hbar, double *cs, double *sn, double *g, double *out);
void arnoldi_post(hipStream_t s, int j, int m, const double *h1, const double *h2,
                  const double *hn2, double *Hbar, double *cs, double *sn, double *g,
                  double *out);
void g_init(hipStream_t s, int m, const double *beta2, double *g, double *beta);
void upper_solve(hipStream_t s, int k, int m, const double *Hbar, const double *g, double *sv);
void rhs_assemble(hipStream_t s, int N, int M, int Nc, const double *us, const double *F,
                  const double *B, double *b);

// Learned body mobility network (mlp.hip)
int64_t mlp_workspace_bytes(int Bp);
int64_t mlp_param_bytes();
int mlp_n_params();
void mlp_refresh(hipStream_t s, void *params);
float *mlp_forward(hipStream_t s, void *params, void *ws, int n, int Bp, const float *X);
int mlp_backward(hipStream_t s, void *params, void *ws, int n, int Bp, const float *X,
                 const float *T, double **lpart);
void mlp_adam(hipStream_t s, void *params, float lr, int t);
void mlp_features(hipStream_t s, int M, const double *q, const double *theta, const int *type,
                  double a, float *X);
void mlp_mobility(hipStream_t s, void *params, int M, const float *Y, double a, double eta,
                  double *Nt, int *bad);
int64_t mlp_state_bytes();
void mlp_set_scaling(hipStream_t s, void *params, const float *in_mu, const float *in_sd,
                     const float *out_mu, const float *out_sd);
void mlp_destandardize(hipStream_t s, void *params, int n, float *Y);
void mlp_targets(hipStream_t s, int M, const double *Nt, double a, double eta, float *T, int *bad);

// Position correction (Sec. 4.2, App. B)
struct CorrectDev {
    int A = 0, M = 0, P = 0;
    const int *asm_body_ptr = nullptr, *asm_bodies = nullptr;
    const int *asm_link_ptr = nullptr, *asm_links = nullptr;
    const int *local_index = nullptr;   // body -> index inside its assembly
    const int *pq = nullptr;
    const double *dl_p = nullptr, *dl_q = nullptr;
    const int64_t *ws_off = nullptr;     // per assembly workspace offsets (doubles)
    double *ws = nullptr;
    double *q = nullptr, *theta = nullptr;
    int *iters = nullptr;
    double *resid = nullptr;
};
void correct_positions(hipStream_t s, const CorrectDev &C, double tol, int max_iter);

// Single-blob bodies (Sec. 2.4): generalised RPY product (rot_pair.hip), the
// self-mobility blocks N~ and the preconditioner apply for y = [U; phi]
int rot_pair_slices(int M);
// work / n_work: the symmetric form on that work list (pair_sym_worklist of M
// bodies), NULL: the target-parallel form; partial holds rot_pair_slices(M) x 6M
// doubles (6M for the symmetric form)
void rot_pair_apply(hipStream_t s, int precision, int M, const double4 *p64, const float4 *hi,
                    const float4 *lo, const double *x6, double a, double scale,
                    const double *base, double *partial, double *out, const int4 *work,
                    int n_work);
// out_i = base_i + (scale_u u_i, scale_w w_i) from one 6 x M partial sum
void rot_reduce(hipStream_t s, int M, const double *partial, double scale_u, double scale_w,
                const double *base, double *out);
void single_blob_body_mobility(hipStream_t s, int M, double a, double eta, double *Nt);
void precond_apply_single(hipStream_t s, const PrecondDev &P, const int *zero_off,
                          const int64_t *zero_off64, const double *r, double *z);

// Reconstruction of articulated bodies from their orientations (Sec. 4.1) and
// the link residual.  Articulated bodies (bodies joined by links) are listed
// as in CorrectDev; per body (by position in asm_bodies) a CSR list of its
// links: entry 2 e + s, e the link's position inside its articulated body's
// link list, s = 1 when the body is the link's - end.
struct ReconDev {
    int A = 0;
    const int *asm_body_ptr = nullptr, *asm_bodies = nullptr;
    const int *asm_link_ptr = nullptr, *asm_links = nullptr;
    const int *adj_ptr = nullptr, *adj = nullptr;
    const int *pq = nullptr;
    const int *anchored = nullptr;       // per articulated body: has a link to a lab point
    const int64_t *g_off = nullptr;      // per articulated body: offset of G (doubles)
    const double *G = nullptr;           // M_a x M_a row-major per articulated body
    const double *dl_p = nullptr, *dl_q = nullptr, *theta = nullptr;
    double *q = nullptr;
    double *z = nullptr;                 // 3 per link (by position in asm_links)
    double *b = nullptr;                 // 3 per body (by position in asm_bodies)
    double *ginf = nullptr, *g2 = nullptr;  // per articulated body
};
// rebuild != 0: q <- reconstruction, then the residual; rebuild == 0: residual only
void reconstruct(hipStream_t s, const ReconDev &D, int rebuild);

}  // namespace arb

// ---------------------------------------------------------------- context
// HIP graphs of the GMRES iteration, one per Arnoldi index j >= 1, valid for
// the key they were captured under
constexpr int kPinnedScalars = 64;
constexpr int kPinnedTotal = kPinnedScalars + 2 * 260;

struct GmresGraphs {
    std::vector<hipGraphExec_t> exec;
    std::vector<long long> key;
    bool broken = false;  // a capture failed: plain launches from then on
    void clear() {
        for (auto &e : exec)
            if (e) (void)hipGraphExecDestroy(e);
        exec.clear();
        key.clear();
    }
    GmresGraphs() = default;
    GmresGraphs(const GmresGraphs &) = delete;
    GmresGraphs &operator=(const GmresGraphs &) = delete;
    ~GmresGraphs() { clear(); }
};

struct arb_ctx {
    arb_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    // bodies
    int N = 0, M = 0;
    std::vector<int> h_blob_off, h_body_of_blob, h_body_type;
    std::vector<double> h_r_ref;
    bool have_state = false;
    // constraints (host copies)
    int P = 0, Rg = 0, Nc = 0;
    std::vector<int> h_pq, h_nproj, h_gpq;
    std::vector<double> h_dl_p, h_dl_q, h_dldot_p, h_dldot_q, h_proj, h_gcoef, h_grhs;
    bool topo_dirty = true;
    int n_asm = 0;
    int max_m = 0;
    std::vector<int> h_asm_body_ptr, h_asm_bodies, h_asm_row_ptr, h_asm_rows;
    // autotune cache: key = N*4 + precision*2 + wall -> launch shape; values > 0
    // are source slices of the target-parallel kernel, values < 0 select the
    // symmetric kernel with -value source tiles per work item
    std::map<int64_t, int> slice_cache;
    // symmetric-kernel work lists, one per precision [ARB_FP64, ARB_FP32C] (each
    // keyed by size and tiles per item), so that a graph captured for one
    // precision never reads a list rebuilt for the other
    arb::DevBuf sym_work[2];
    int sym_work_N[2] = {-1, -1}, sym_work_R[2] = {-1, -1};
    int sym_n_work[2] = {0, 0};
    bool pc_built = false;
    bool pc_learned = false;
    bool pc_lcorr = false;  // learned body mobility with the consistent blob-block correction
    int pc_pinv = 0;

    // device buffers
    arb::DevBuf blob_off, body_of_blob, r_ref, q, theta, R9, pos, dvec, p64, hi, lo,
        partial, row_p, row_q, row_kind, row_src, row_m, dl_p, dl_q, dldot_p, dldot_q, proj,
        gcoef, grhs, crow, Bc, brow_ptr, brow_ent, asm_body_ptr, asm_bodies, asm_row_ptr,
        asm_rows, asm_mat_off, mat_off, z_off, mats, minv, ldiag, dinv, Z, Nt, G, S, status, pctmp, lcorr, stmp,
        asm_dinv, asm_fail, body_pinv;
    int asm_max_rows = 0;  // largest assembly (constraint rows)
    int n_brow_ent = 0;    // entries of the bodies' constraint-row lists
    // generic scratch for host entry points and the solver
    arb::DevBuf s_in, s_out, s_aux, s_pos;
    arb::DevBuf tbox;  // per 64-blob tile of the state's positions: bounding box (prep_positions)
    // the dense pair kernels' copy of the state's positions in Morton order when the
    // blobs' own order leaves tiles spread out (pair_order in api.hip): the
    // permutation (entry k = blob pperm[k]), positions and tile boxes in that order
    bool psorted = false;
    arb::DevBuf pperm, p64s, his, los, tboxs;
    arb::DevBuf kv, kH, kcs, ksn, kg, khcol, khn, ksv, kpart, kb, kr, kz, kw, ky, kt, ksteps;
    // host pinned scratch: kPinnedScalars doubles for entry points, then two per
    // Arnoldi step (h_{j+1,j}, residual estimate) at pinned + kPinnedScalars
    double *pinned = nullptr;
    // one event per Arnoldi step of a cycle: the host waits on step j's scalars
    // while later steps may already run
    std::vector<hipEvent_t> step_ev;
    GmresGraphs ggraph;
    // articulated bodies (bodies joined by links) for the correction and the
    // reconstruction, rebuilt when bodies or links change
    bool lasm_dirty = true;
    int lasm_A = 0;
    int64_t lasm_ws = 0;   // correction workspace (doubles)
    bool lasm_fits_corr = true;
    arb::DevBuf c_link_ptr, c_links, c_local, c_ws_off, c_ws, c_iters, c_resid, c_pq, c_abp, c_ab;
    arb::DevBuf r_adj_ptr, r_adj, r_anch, r_goff, r_G, r_z, r_b, r_ginf, r_g2;
    // last solution of a solve (warm start of the next time step); ky_n = its length
    int64_t ky_n = 0;
    // single-blob model: M+1 zero offsets (no blobs in the preconditioner's body
    // stage), partial sums of the generalised RPY product, C^T phi
    arb::DevBuf zero_off, zero_off64, rot_partial, rot_ct, rot_work;
    int rot_work_M = -1, rot_n_work = 0;
    // the initial state of a midpoint step
    arb::DevBuf q0, th0;
    arb::DevBuf tune_out;
    // learned body mobility: network parameters, workspace, per-type blocks
    arb::DevBuf mlp_params, mlp_ws, mlp_x, mlp_t, body_type_d, t_ref, t_mat_off, t_z_off, t_minv,
        t_Z, t_mats, t_ldiag, t_dinv, t_Nt, t_blob_off, t_status, t_body_pinv;
    bool mlp_ready = false;
    int mlp_step = 0;
    bool types_ready = false;
    std::vector<int> h_type_ref;  // reference body of each type
    // fast product (ARB_PAIR_FMM)
    arb::FmmState fmm;
    // pair-kernel timing (arb_profile)
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
};
