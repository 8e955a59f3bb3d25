// C ABI of libarb (declared in include/arb.h): argument checking, topology
// bookkeeping on the host, and launch orchestration.  Every arithmetic step of
// the method runs in the HIP kernels of pair.hip, bodies.hip, precond.hip,
// krylov.hip and correct.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"

namespace arb {
int64_t correct_ws_doubles(int nb, int nl);
}

using arb::DevBuf;

namespace {

constexpr int kMaxBodyBlobs = 512;
constexpr int kMaxAsmRows = 2048;
constexpr int kMaxCorrRows = 2048;
// largest articulated body (in bodies) the reconstruction takes: G is M_a^2 doubles
constexpr int kMaxReconBodies = 2048;
// FP32 refinement: factor by which the FP32 product's error on the previous
// correction (relative to its right-hand side) is inflated when it stands in
// for the error on the last correction
constexpr double kRefineSafety = 10.0;

// lower Cholesky factor of a symmetric positive definite n x n row-major matrix,
// in place in the lower triangle (the upper one is left as it was); nonzero if
// a pivot is not positive
static int host_cholesky(double *A, int n) {
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0.0)) return 1;
        const double ljj = std::sqrt(d);
        A[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = v / ljj;
        }
    }
    return 0;
}

// in-place inverse of a symmetric positive definite n x n row-major matrix by
// Cholesky (A = C C^T, A^-1 = C^-T C^-1); returns nonzero if not SPD
static int spd_inverse(double *A, int n) {
    std::vector<double> C((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= C[(size_t)j * n + k] * C[(size_t)j * n + k];
        if (!(d > 0.0)) return 1;
        const double cjj = std::sqrt(d);
        C[(size_t)j * n + j] = cjj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= C[(size_t)i * n + k] * C[(size_t)j * n + k];
            C[(size_t)i * n + j] = v / cjj;
        }
    }
    // W = C^-1 (lower), then A^-1 = W^T W
    std::vector<double> W((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        W[(size_t)j * n + j] = 1.0 / C[(size_t)j * n + j];
        for (int i = j + 1; i < n; ++i) {
            double v = 0.0;
            for (int k = j; k < i; ++k) v -= C[(size_t)i * n + k] * W[(size_t)k * n + j];
            W[(size_t)i * n + j] = v / C[(size_t)i * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = 0.0;
            for (int k = i; k < n; ++k) v += W[(size_t)k * n + i] * W[(size_t)k * n + j];
            A[(size_t)i * n + j] = v;
            A[(size_t)j * n + i] = v;
        }
    return 0;
}

int fail(arb_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, ARB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)                 \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ < 0) return rc_;  \
    } while (0)

hipStream_t pick(arb_ctx *ctx, void *stream) {
    return stream ? (hipStream_t)stream : ctx->stream;
}

template <class T>
int upload(arb_ctx *ctx, DevBuf &b, const T *h, size_t n, hipStream_t s) {
    HIPCHK(b.ensure(n * sizeof(T)));
    if (n) HIPCHK(hipMemcpyAsync(b.p, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    return 0;
}

int64_t n_unknowns(const arb_ctx *ctx) {
    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB) return 6 * (int64_t)ctx->M + ctx->Nc;
    return 3 * (int64_t)ctx->N + 6 * (int64_t)ctx->M + ctx->Nc;
}

// M+1 zero blob offsets for the single-blob model (stages written for blobs run
// with none)
static int ensure_zero_offsets(arb_ctx *ctx, hipStream_t s) {
    const size_t want = (size_t)(ctx->M + 1);
    if (ctx->zero_off.bytes >= want * sizeof(int) && ctx->zero_off64.bytes >= want * sizeof(int64_t))
        return 0;
    std::vector<int> z(want, 0);
    std::vector<int64_t> z64(want, 0);
    TRY(upload(ctx, ctx->zero_off, z.data(), want, s));
    TRY(upload(ctx, ctx->zero_off64, z64.data(), want, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

// offset of U inside the solution vector
static int64_t u_offset(const arb_ctx *ctx) {
    return ctx->opt.model == ARB_MODEL_SINGLE_BLOB ? 0 : 3 * (int64_t)ctx->N;
}

// ---------------------------------------------------------------- topology
int build_topology(arb_ctx *ctx) {
    if (!ctx->topo_dirty) return 0;
    const int M = ctx->M;
    hipStream_t s = ctx->stream;
    // constraint row table: link rows (link order, nproj each), then general rows
    std::vector<int> rp, rq, rk, rs, rm;
    for (int n = 0; n < ctx->P; ++n)
        for (int m = 0; m < ctx->h_nproj[n]; ++m) {
            rp.push_back(ctx->h_pq[2 * n]);
            rq.push_back(ctx->h_pq[2 * n + 1]);
            rk.push_back(0);
            rs.push_back(n);
            rm.push_back(m);
        }
    for (int j = 0; j < ctx->Rg; ++j) {
        rp.push_back(ctx->h_gpq[2 * j]);
        rq.push_back(ctx->h_gpq[2 * j + 1]);
        rk.push_back(1);
        rs.push_back(j);
        rm.push_back(0);
    }
    const int Nc = (int)rp.size();
    ctx->Nc = Nc;
    for (int k = 0; k < Nc; ++k)
        if (rp[k] < 0 || rp[k] >= M || rq[k] < -1 || rq[k] >= M || rq[k] == rp[k])
            return fail(ctx, ARB_E_ARG, "constraint refers to a body outside 0..M-1");
    // per-body CSR of (row, side) entries for C^T phi, rows ascending
    std::vector<int> bptr(M + 1, 0), bent;
    for (int k = 0; k < Nc; ++k) {
        bptr[rp[k] + 1]++;
        if (rq[k] >= 0) bptr[rq[k] + 1]++;
    }
    for (int p = 0; p < M; ++p) bptr[p + 1] += bptr[p];
    bent.assign(bptr[M], 0);
    std::vector<int> fill(bptr.begin(), bptr.end() - 1);
    for (int k = 0; k < Nc; ++k) {
        bent[fill[rp[k]]++] = 2 * k;
        if (rq[k] >= 0) bent[fill[rq[k]]++] = 2 * k + 1;
    }
    // assemblies: union of bodies joined by any row
    std::vector<int> parent(M);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int i) {
        while (parent[i] != i) {
            parent[i] = parent[parent[i]];
            i = parent[i];
        }
        return i;
    };
    for (int k = 0; k < Nc; ++k)
        if (rq[k] >= 0) {
            int a = find(rp[k]), b = find(rq[k]);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    std::vector<int> label(M, -1), asm_of(M);
    int A = 0;
    for (int p = 0; p < M; ++p) {
        const int r = find(p);
        if (label[r] < 0) label[r] = A++;
        asm_of[p] = label[r];
    }
    std::vector<int> abp(A + 1, 0), ab(M), arp(A + 1, 0), ar(Nc);
    for (int p = 0; p < M; ++p) abp[asm_of[p] + 1]++;
    for (int a = 0; a < A; ++a) abp[a + 1] += abp[a];
    {
        std::vector<int> f2(abp.begin(), abp.end() - 1);
        for (int p = 0; p < M; ++p) ab[f2[asm_of[p]]++] = p;
    }
    for (int k = 0; k < Nc; ++k) arp[asm_of[rp[k]] + 1]++;
    for (int a = 0; a < A; ++a) arp[a + 1] += arp[a];
    {
        std::vector<int> f2(arp.begin(), arp.end() - 1);
        for (int k = 0; k < Nc; ++k) ar[f2[asm_of[rp[k]]]++] = k;
    }
    std::vector<int64_t> amo(A + 1, 0);
    for (int a = 0; a < A; ++a) {
        const int na = arp[a + 1] - arp[a];
        if (na > kMaxAsmRows)
            return fail(ctx, ARB_E_ARG, "articulated body with more than 2048 constraint rows");
        amo[a + 1] = amo[a] + (int64_t)na * na;
    }
    ctx->n_asm = A;
    ctx->h_asm_body_ptr = abp;
    ctx->h_asm_bodies = ab;
    ctx->h_asm_row_ptr = arp;
    ctx->h_asm_rows = ar;
    TRY(upload(ctx, ctx->row_p, rp.data(), Nc, s));
    TRY(upload(ctx, ctx->row_q, rq.data(), Nc, s));
    TRY(upload(ctx, ctx->row_kind, rk.data(), Nc, s));
    TRY(upload(ctx, ctx->row_src, rs.data(), Nc, s));
    TRY(upload(ctx, ctx->row_m, rm.data(), Nc, s));
    TRY(upload(ctx, ctx->brow_ptr, bptr.data(), M + 1, s));
    TRY(upload(ctx, ctx->brow_ent, bent.data(), bent.size(), s));
    ctx->n_brow_ent = (int)bent.size();
    TRY(upload(ctx, ctx->asm_body_ptr, abp.data(), A + 1, s));
    TRY(upload(ctx, ctx->asm_bodies, ab.data(), M, s));
    TRY(upload(ctx, ctx->asm_row_ptr, arp.data(), A + 1, s));
    TRY(upload(ctx, ctx->asm_rows, ar.data(), Nc, s));
    TRY(upload(ctx, ctx->asm_mat_off, amo.data(), A + 1, s));
    HIPCHK(ctx->G.ensure(std::max<int64_t>(amo[A], 1) * sizeof(double)));
    HIPCHK(ctx->S.ensure(std::max<int64_t>(2 * amo[A], 1) * sizeof(double)));
    // the blocked factorisation of the assemblies' S_a: diagonal-block inverses
    // (1,024 doubles per 32-row block) and a failure flag per assembly
    ctx->asm_max_rows = 0;
    for (int a = 0; a < A; ++a) ctx->asm_max_rows = std::max(ctx->asm_max_rows, arp[a + 1] - arp[a]);
    HIPCHK(ctx->asm_dinv.ensure(std::max<int64_t>(32 * (int64_t)Nc + 1024 * (int64_t)A, 1) *
                                sizeof(double)));
    HIPCHK(ctx->asm_fail.ensure(std::max(A, 1) * sizeof(int)));
    HIPCHK(ctx->crow.ensure(std::max(Nc, 1) * 12 * sizeof(double)));
    HIPCHK(ctx->Bc.ensure(std::max(Nc, 1) * sizeof(double)));
    // link data (zero-size arrays still get a valid pointer)
    const int P = ctx->P;
    TRY(upload(ctx, ctx->dl_p, ctx->h_dl_p.data(), 3 * (size_t)P, s));
    TRY(upload(ctx, ctx->dl_q, ctx->h_dl_q.data(), 3 * (size_t)P, s));
    TRY(upload(ctx, ctx->dldot_p, ctx->h_dldot_p.data(), 3 * (size_t)P, s));
    TRY(upload(ctx, ctx->dldot_q, ctx->h_dldot_q.data(), 3 * (size_t)P, s));
    TRY(upload(ctx, ctx->proj, ctx->h_proj.data(), 9 * (size_t)P, s));
    TRY(upload(ctx, ctx->gcoef, ctx->h_gcoef.data(), 12 * (size_t)ctx->Rg, s));
    TRY(upload(ctx, ctx->grhs, ctx->h_grhs.data(), (size_t)ctx->Rg, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->topo_dirty = false;
    ctx->pc_built = false;
    return 0;
}

int refresh_rows(arb_ctx *ctx, hipStream_t s) {
    if (ctx->Nc > 0)
        arb::constraint_rows(s, ctx->Nc, ctx->row_p.as<int>(), ctx->row_q.as<int>(),
                             ctx->row_kind.as<int>(), ctx->row_src.as<int>(), ctx->row_m.as<int>(),
                             ctx->R9.as<double>(), ctx->dl_p.as<double>(), ctx->dl_q.as<double>(),
                             ctx->dldot_p.as<double>(), ctx->dldot_q.as<double>(),
                             ctx->proj.as<double>(), ctx->gcoef.as<double>(),
                             ctx->grhs.as<double>(), ctx->crow.as<double>(), ctx->Bc.as<double>());
    return 0;
}

int ready(arb_ctx *ctx) {
    if (ctx->M <= 0) return fail(ctx, ARB_E_ARG, "bodies not set");
    if (!ctx->have_state) return fail(ctx, ARB_E_ARG, "state not set");
    if (ctx->topo_dirty) {
        TRY(build_topology(ctx));
        TRY(refresh_rows(ctx, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return 0;
}

// 21 bits of x spread to every third bit (Morton interleaving)
uint64_t spread21(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// The dense pair kernels' blob order for the current state.  The symmetric FP32
// kernel tests tiles of 64 consecutive blobs for distance; when the blobs' own
// order leaves tiles spread over the suspension (loose blobs in random order:
// mean tile diagonal above a quarter of the suspension's), the products run on
// a copy sorted along a Morton curve, made here once per state (positions and
// tile boxes in that order, and the permutation, through which the kernels read
// lambda and write u).  Bodies' blobs, contiguous per body, already give compact
// tiles and keep their order.
int pair_order(arb_ctx *ctx, hipStream_t s) {
    const int N = ctx->N;
    const int nt = (N + 63) / 64;
    ctx->psorted = false;
    // only the dense multiblob products read the sorted copy
    if (nt < 8 || ctx->opt.model == ARB_MODEL_SINGLE_BLOB || ctx->opt.pair_kernel == ARB_PAIR_FMM)
        return 0;
    std::vector<float4> box(2 * (size_t)nt);
    HIPCHK(hipMemcpyAsync(box.data(), ctx->tbox.p, box.size() * sizeof(float4),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float lo[3] = {box[0].x, box[0].y, box[0].z}, hi[3] = {box[1].x, box[1].y, box[1].z};
    double mean = 0.0;
    for (int t = 0; t < nt; ++t) {
        const float4 a = box[2 * t], b = box[2 * t + 1];
        lo[0] = std::min(lo[0], a.x), lo[1] = std::min(lo[1], a.y), lo[2] = std::min(lo[2], a.z);
        hi[0] = std::max(hi[0], b.x), hi[1] = std::max(hi[1], b.y), hi[2] = std::max(hi[2], b.z);
        mean += std::sqrt(double(b.x - a.x) * (b.x - a.x) + double(b.y - a.y) * (b.y - a.y) +
                          double(b.z - a.z) * (b.z - a.z));
    }
    mean /= nt;
    // the diagonal of a compact tile: a cube holding 64 blobs at the domain's mean
    // density (positions in units of a); sort when the tiles as given are much
    // larger (random order, or bodies whose tiles straddle distant bodies)
    double vol = 1.0;
    for (int c = 0; c < 3; ++c) vol *= std::max(double(hi[c] - lo[c]), 2.0);
    const double compact = std::sqrt(3.0) * std::cbrt(64.0 * vol / N);
    if (!(mean > 2.0 * compact)) return 0;
    std::vector<double> pos(3 * (size_t)N);
    HIPCHK(hipMemcpyAsync(pos.data(), ctx->pos.p, pos.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double pl[3], ph[3];
    for (int c = 0; c < 3; ++c) pl[c] = ph[c] = pos[c];
    for (int i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            pl[c] = std::min(pl[c], pos[3 * (size_t)i + c]);
            ph[c] = std::max(ph[c], pos[3 * (size_t)i + c]);
        }
    const double side = std::max({ph[0] - pl[0], ph[1] - pl[1], ph[2] - pl[2], 1e-300});
    std::vector<std::pair<uint64_t, int>> key((size_t)N);
    for (int i = 0; i < N; ++i) {
        uint64_t k = 0;
        for (int c = 0; c < 3; ++c) {
            const double f = (pos[3 * (size_t)i + c] - pl[c]) / side;
            const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, f * 2097151.0));
            k |= spread21(q) << (2 - c);
        }
        key[i] = {k, i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> perm((size_t)N);
    for (int k = 0; k < N; ++k) perm[k] = key[k].second;
    TRY(upload(ctx, ctx->pperm, perm.data(), N, s));
    HIPCHK(ctx->p64s.ensure((size_t)N * sizeof(double4)));
    HIPCHK(ctx->his.ensure((size_t)N * sizeof(float4)));
    HIPCHK(ctx->los.ensure((size_t)N * sizeof(float4)));
    HIPCHK(ctx->tboxs.ensure(2 * (size_t)nt * sizeof(float4)));
    // the sorted copy is centred in x and y: smaller |x| lets more tile pairs take
    // the far path (its criterion scales with the largest |coordinate|)
    arb::prep_positions(s, N, ctx->pos.as<double>(), ctx->opt.a, ctx->p64s.as<double4>(),
                        ctx->his.as<float4>(), ctx->los.as<float4>(), ctx->tboxs.as<float4>(),
                        ctx->pperm.as<int>(), 0.5 * (pl[0] + ph[0]), 0.5 * (pl[1] + ph[1]));
    ctx->psorted = true;
    return 0;
}

// geometry of the current state: rotations, blob positions, constraint rows
int refresh_geometry(arb_ctx *ctx, hipStream_t s) {
    const int N = ctx->N, M = ctx->M;
    HIPCHK(ctx->R9.ensure(9 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->pos.ensure(3 * (size_t)N * sizeof(double)));
    HIPCHK(ctx->dvec.ensure(3 * (size_t)N * sizeof(double)));
    HIPCHK(ctx->p64.ensure((size_t)N * sizeof(double4)));
    HIPCHK(ctx->hi.ensure((size_t)N * sizeof(float4)));
    HIPCHK(ctx->lo.ensure((size_t)N * sizeof(float4)));
    HIPCHK(ctx->tbox.ensure(2 * (size_t)std::max((N + 63) / 64, 1) * sizeof(float4)));
    arb::rotations(s, M, ctx->theta.as<double>(), ctx->R9.as<double>());
    arb::blob_geometry(s, N, ctx->body_of_blob.as<int>(), ctx->q.as<double>(), ctx->R9.as<double>(),
                       ctx->r_ref.as<double>(), ctx->pos.as<double>(), ctx->dvec.as<double>());
    arb::prep_positions(s, N, ctx->pos.as<double>(), ctx->opt.a, ctx->p64.as<double4>(),
                        ctx->hi.as<float4>(), ctx->lo.as<float4>(), ctx->tbox.as<float4>(),
                        nullptr);
    TRY(pair_order(ctx, s));
    if (!ctx->topo_dirty) TRY(refresh_rows(ctx, s));
    ctx->pc_built = false;
    ctx->fmm.dirty = true;
    return 0;
}

// ---------------------------------------------------------------- pair launch
using arb::heuristic_slices;

int sym_worklist(arb_ctx *ctx, hipStream_t s, int N, int R, int precision) {
    const int pi = precision == ARB_FP32C ? 1 : 0;
    if (ctx->sym_work_N[pi] == N && ctx->sym_work_R[pi] == R) return 0;
    std::vector<int4> w = arb::pair_sym_worklist(N, R);
    HIPCHK(ctx->sym_work[pi].ensure(std::max<size_t>(w.size(), 1) * sizeof(int4)));
    if (!w.empty())
        HIPCHK(hipMemcpyAsync(ctx->sym_work[pi].p, w.data(), w.size() * sizeof(int4),
                              hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->sym_work_N[pi] = N;
    ctx->sym_work_R[pi] = R;
    ctx->sym_n_work[pi] = (int)w.size();
    return 0;
}

// one pair product; shape > 0: target-parallel kernel with that many source
// slices; shape < 0: symmetric kernel with -shape source tiles per work item
int run_pair(arb_ctx *ctx, hipStream_t s, int N, const double4 *p64, const float4 *hi,
             const float4 *lo, const float4 *box, const int *perm, const double *lam, double *out,
             const double *U, const int *bob,
             const double *dvec, int precision, bool wall, int shape) {
    const bool sym = shape < 0;
    // small systems take the run-sliced target-parallel kernel whatever the shape
    const bool small = N <= arb::kSmallPairN && ctx->opt.pair_kernel != ARB_PAIR_SYMMETRIC;
    int used = 1;
    if (small) {
        const int runs = (N + arb::kSmallRun - 1) / arb::kSmallRun;
        HIPCHK(ctx->partial.ensure((size_t)runs * 3 * N * sizeof(double)));
    } else if (sym) {
        TRY(sym_worklist(ctx, s, N, -shape, precision));
        HIPCHK(ctx->partial.ensure((size_t)3 * N * sizeof(double)));
    } else {
        HIPCHK(ctx->partial.ensure((size_t)shape * 3 * N * sizeof(double)));
    }
    if (sym && !small) arb::pair_sym_clear(s, N, ctx->partial.as<double>());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->prof) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
    }
    if (small)
        used = arb::pair_partial_small(s, precision, wall, N, p64, hi, lo, lam, perm, ctx->opt.a,
                                       ctx->partial.as<double>());
    else if (sym)
        arb::pair_sym(s, precision, wall, N, p64, hi, lo, box, lam, perm, ctx->opt.a,
                      ctx->sym_work[precision == ARB_FP32C].as<int4>(),
                      ctx->sym_n_work[precision == ARB_FP32C], ctx->partial.as<double>());
    else
        used = arb::pair_partial(s, precision, wall, N, p64, hi, lo, lam, perm, ctx->opt.a, shape,
                                 ctx->partial.as<double>());
    if (ctx->prof) {
        HIPCHK(hipEventRecord(e1, s));
        ctx->prof_ev.emplace_back(e0, e1);
    }
    // FP32 sums are in units of the blob radius: M(a) = M_{a=1}(r / a) / a
    const double scale = 1.0 / (8.0 * arb::kPi * ctx->opt.eta) /
                         (precision == ARB_FP32C ? ctx->opt.a : 1.0);
    arb::pair_reduce(s, N, used, ctx->partial.as<double>(), scale, out, U, bob, dvec, perm);
    return 0;
}

// launch shape for (N, precision, wall): from the options, the cache, or by
// timing every candidate shape on the first product of that size
int choose_slices(arb_ctx *ctx, hipStream_t s, int N, const double4 *p64, const float4 *hi,
                  const float4 *lo, const float4 *box, const int *perm, const double *lam,
                  int precision, bool wall, int *shape) {
    const int kind = ctx->opt.pair_kernel;
    const bool sym_ok = kind != 1;
    if (ctx->opt.slices > 0 && kind != 2) {
        *shape = ctx->opt.slices;
        return 0;
    }
    const int64_t key = (int64_t)N * 4 + precision * 2 + (wall ? 1 : 0);
    auto it = ctx->slice_cache.find(key);
    if (it != ctx->slice_cache.end()) {
        *shape = it->second;
        return 0;
    }
    const int h = heuristic_slices(N);
    const int ntiles = (N + arb::kTile - 1) / arb::kTile;
    std::vector<int> cand;
    // from 65,536 blobs the heuristic slice count alone stands for the
    // target-parallel kernel (it fills the chip with one slice or two)
    if (kind != 2) {
        if (N >= 65536)
            cand.push_back(h);
        else
            for (int c = std::max(1, h / 2); c <= std::min(ntiles, h * 16); c *= 2)
                cand.push_back(c);
    }
    if (sym_ok)
        for (int R : {1, 2, 4, 8, 16}) cand.push_back(-R);
    int best = cand.empty() ? h : cand[0];
    if (N >= 8192 && cand.size() > 1) {
        HIPCHK(ctx->tune_out.ensure(3 * (size_t)N * sizeof(double)));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // the fastest of up to 4 timed runs per shape (after one untimed), so
        // that a single slow run does not decide; products of more than 20 ms
        // vary little between runs and are timed once
        float bt = 1e30f;
        for (int c : cand) {
            float tmin = 1e30f;
            for (int rep = 0, reps = 5; rep < reps; ++rep) {
                HIPCHK(hipEventRecord(e0, s));
                TRY(run_pair(ctx, s, N, p64, hi, lo, box, perm, lam, ctx->tune_out.as<double>(),
                             nullptr, nullptr, nullptr, precision, wall, c));
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (rep == 0 && ms > 20.f) reps = 2;
                if (rep > 0) tmin = std::min(tmin, ms);
            }
            if (tmin < bt) {
                bt = tmin;
                best = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } else if (sym_ok && kind == 2) {
        best = -4;
    }
    ctx->slice_cache[key] = best;
    *shape = best;
    return 0;
}

// the fast product (ARB_PAIR_FMM): the tree is rebuilt when the geometry has
// changed (or when asked), then out = M lambda - K U as run_pair writes it
int fmm_pair(arb_ctx *ctx, hipStream_t s, int N, const double *pos, const float4 *hi,
             const float4 *lo, const double *lam, double *out, const double *U, const int *bob,
             const double *dvec, bool rebuild, int precision) {
    arb::FmmState &F = ctx->fmm;
    if (rebuild || F.dirty || !F.ready || F.N != N) {
        std::string msg;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = arb::fmm_build(F, s, N, pos, hi, lo, ctx->opt.a, ctx->opt.fmm_order,
                                      ctx->opt.fmm_levels, ctx->opt.fmm_leaf, 1, &msg);
        if (rc) return fail(ctx, rc, msg);
        F.build_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
        F.dirty = false;
    }
    HIPCHK(ctx->partial.ensure((size_t)3 * std::max(N, 1) * sizeof(double)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->prof) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
    }
    arb::fmm_apply(F, s, ctx->opt.wall != 0, precision == ARB_FP64, lam,
                   ctx->partial.as<double>());
    if (ctx->prof) {
        HIPCHK(hipEventRecord(e1, s));
        ctx->prof_ev.emplace_back(e0, e1);
    }
    // sums in units of the blob radius: M(a) = M_{a=1}(r / a) / a
    const double scale = 1.0 / (8.0 * arb::kPi * ctx->opt.eta) / ctx->opt.a;
    if (N > 0)
        arb::pair_reduce(s, N, 1, ctx->partial.as<double>(), scale, out, U, bob, dvec, nullptr);
    return 0;
}

int ctx_pair(arb_ctx *ctx, hipStream_t s, const double *lam, double *out, const double *U,
             int precision) {
    if (ctx->opt.pair_kernel == ARB_PAIR_FMM)
        return fmm_pair(ctx, s, ctx->N, ctx->pos.as<double>(), ctx->hi.as<float4>(),
                        ctx->lo.as<float4>(), lam, out, U, ctx->body_of_blob.as<int>(),
                        ctx->dvec.as<double>(), false, precision);
    const bool wall = ctx->opt.wall != 0;
    // the state's positions in the pair kernels' order (pair_order)
    const bool so = ctx->psorted;
    const double4 *p64 = (so ? ctx->p64s : ctx->p64).as<double4>();
    const float4 *hi = (so ? ctx->his : ctx->hi).as<float4>();
    const float4 *lo = (so ? ctx->los : ctx->lo).as<float4>();
    const float4 *box = (so ? ctx->tboxs : ctx->tbox).as<float4>();
    const int *perm = so ? ctx->pperm.as<int>() : nullptr;
    int sl = 0;
    TRY(choose_slices(ctx, s, ctx->N, p64, hi, lo, box, perm, lam, precision, wall, &sl));
    return run_pair(ctx, s, ctx->N, p64, hi, lo, box, perm, lam, out, U,
                    ctx->body_of_blob.as<int>(), ctx->dvec.as<double>(), precision, wall, sl);
}

// out = A y (Eq. linear_system)
int single_blob_system_apply(arb_ctx *ctx, hipStream_t s, const double *y, double *out,
                             int precision);

int system_apply(arb_ctx *ctx, hipStream_t s, const double *y, double *out, int precision) {
    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB)
        return single_blob_system_apply(ctx, s, y, out, precision);
    const int N = ctx->N, M = ctx->M;
    const double *lam = y, *U = y + 3 * (size_t)N, *phi = y + 3 * (size_t)N + 6 * (size_t)M;
    TRY(ctx_pair(ctx, s, lam, out, U, precision));
    arb::KT_CT_apply(s, M, ctx->blob_off.as<int>(), ctx->dvec.as<double>(), lam, -1.0,
                     ctx->brow_ptr.as<int>(), ctx->brow_ent.as<int>(), ctx->crow.as<double>(),
                     ctx->Nc > 0 ? phi : nullptr, out + 3 * (size_t)N);
    arb::C_apply(s, ctx->Nc, ctx->row_p.as<int>(), ctx->row_q.as<int>(), ctx->crow.as<double>(), U,
                 out + 3 * (size_t)N + 6 * (size_t)M);
    return 0;
}

// generalised RPY product N x6 (6M) scaled into out = base + scale' N x6, with the
// kernel's 1/(8 pi eta) folded into scale' = scale / (8 pi eta)
// the symmetric form from 4,096 bodies on (or when the options ask for it): enough
// work items to fill the chip; the target-parallel form below
static bool rot_symmetric(const arb_ctx *ctx) {
    return ctx->opt.pair_kernel == ARB_PAIR_SYMMETRIC ||
           (ctx->opt.pair_kernel == ARB_PAIR_AUTO && ctx->M >= 4096);
}

int body_mobility_dev(arb_ctx *ctx, hipStream_t s, const double *x6, double scale,
                      const double *base, double *out, int precision) {
    const int M = ctx->M;
    if (ctx->opt.pair_kernel == ARB_PAIR_FMM) {
        // the fast product of the generalised tensor: tree of the body positions
        // with a torque channel, rebuilt when the state has changed
        arb::FmmState &F = ctx->fmm;
        if (F.dirty || !F.ready || F.N != M || F.channels < 2) {
            std::string msg;
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = arb::fmm_build(F, s, M, ctx->pos.as<double>(), ctx->hi.as<float4>(),
                                          ctx->lo.as<float4>(), ctx->opt.a, ctx->opt.fmm_order,
                                          ctx->opt.fmm_levels, ctx->opt.fmm_leaf, 2, &msg);
            if (rc) return fail(ctx, rc, msg);
            F.build_ms = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - t0)
                             .count();
            F.dirty = false;
        }
        HIPCHK(ctx->rot_partial.ensure(std::max<int64_t>(6 * (int64_t)M, 1) * sizeof(double)));
        const double a = ctx->opt.a, k = scale / (8.0 * arb::kPi * ctx->opt.eta);
        arb::fmm_apply6(F, s, precision == ARB_FP64, x6, 1.0 / a, ctx->rot_partial.as<double>());
        arb::rot_reduce(s, M, ctx->rot_partial.as<double>(), k / a, k / (a * a), base, out);
        return 0;
    }
    HIPCHK(ctx->rot_partial.ensure(std::max<int64_t>(
        (int64_t)arb::rot_pair_slices(M) * 6 * M, 1) * sizeof(double)));
    const int4 *work = nullptr;
    if (rot_symmetric(ctx)) {
        if (ctx->rot_work_M != M) {
            // built on the first product of a size (the solve's right-hand side), so
            // never inside a captured GMRES step
            std::vector<int4> w = arb::pair_sym_worklist(M, 1);
            HIPCHK(ctx->rot_work.ensure(std::max<size_t>(w.size(), 1) * sizeof(int4)));
            HIPCHK(hipMemcpyAsync(ctx->rot_work.p, w.data(), w.size() * sizeof(int4),
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            ctx->rot_work_M = M;
            ctx->rot_n_work = (int)w.size();
        }
        work = ctx->rot_work.as<int4>();
    }
    const double k = 1.0 / (8.0 * arb::kPi * ctx->opt.eta);
    arb::rot_pair_apply(s, precision, M, ctx->p64.as<double4>(), ctx->hi.as<float4>(),
                        ctx->lo.as<float4>(), x6, ctx->opt.a, scale * k, base,
                        ctx->rot_partial.as<double>(), out, work, ctx->rot_n_work);
    return 0;
}

// y = [U; phi] -> [U - N C^T phi; C U] (Eq. linear_system_general, rows reordered)
int single_blob_system_apply(arb_ctx *ctx, hipStream_t s, const double *y, double *out,
                             int precision) {
    const int M = ctx->M;
    const double *U = y, *phi = y + 6 * (size_t)M;
    HIPCHK(ctx->rot_ct.ensure(6 * (size_t)M * sizeof(double)));
    TRY(ensure_zero_offsets(ctx, s));
    // C^T phi: the balance-row kernel with no blobs
    arb::KT_CT_apply(s, M, ctx->zero_off.as<int>(), ctx->dvec.as<double>(), nullptr, -1.0,
                     ctx->brow_ptr.as<int>(), ctx->brow_ent.as<int>(), ctx->crow.as<double>(),
                     ctx->Nc > 0 ? phi : nullptr, ctx->rot_ct.as<double>());
    TRY(body_mobility_dev(ctx, s, ctx->rot_ct.as<double>(), -1.0, U, out, precision));
    arb::C_apply(s, ctx->Nc, ctx->row_p.as<int>(), ctx->row_q.as<int>(), ctx->crow.as<double>(), U,
                 out + 6 * (size_t)M);
    return 0;
}

arb::PrecondDev pc_view(arb_ctx *ctx) {
    arb::PrecondDev P;
    P.M = ctx->M;
    P.A = ctx->n_asm;
    P.blob_off = ctx->blob_off.as<int>();
    P.mat_off = ctx->mat_off.as<int64_t>();
    P.z_off = ctx->z_off.as<int64_t>();
    P.asm_body_ptr = ctx->asm_body_ptr.as<int>();
    P.asm_bodies = ctx->asm_bodies.as<int>();
    P.asm_row_ptr = ctx->asm_row_ptr.as<int>();
    P.asm_rows = ctx->asm_rows.as<int>();
    P.asm_mat_off = ctx->asm_mat_off.as<int64_t>();
    P.row_p = ctx->row_p.as<int>();
    P.row_q = ctx->row_q.as<int>();
    P.brow_ptr = ctx->brow_ptr.as<int>();
    P.brow_ent = ctx->brow_ent.as<int>();
    P.crow = ctx->crow.as<double>();
    P.mats = ctx->mats.as<double>();
    P.minv = ctx->minv.as<double>();
    P.ldiag = ctx->ldiag.as<double>();
    P.dinv = ctx->dinv.as<double>();
    P.Z = ctx->Z.as<double>();
    P.Nt = ctx->Nt.as<double>();
    P.G = ctx->G.as<double>();
    P.S = ctx->S.as<double>();
    P.asm_max_rows = ctx->asm_max_rows;
    P.asm_dinv = ctx->asm_dinv.as<double>();
    P.asm_fail = ctx->asm_fail.as<int>();
    P.body_pinv = ctx->body_pinv.as<int>();
    P.status = ctx->status.as<int>();
    P.tmp = ctx->pctmp.as<double>();
    P.learned = ctx->pc_learned ? 1 : 0;
    P.type = ctx->body_type_d.as<int>();
    P.tmat_off = ctx->t_mat_off.as<int64_t>();
    P.tz_off = ctx->t_z_off.as<int64_t>();
    P.tminv = ctx->t_minv.as<double>();
    P.tZ = ctx->t_Z.as<double>();
    P.R9 = ctx->R9.as<double>();
    P.lcorr = ctx->pc_lcorr ? ctx->lcorr.as<double>() : nullptr;
    P.stmp = ctx->stmp.as<double>();
    return P;
}

// per-type body-frame unbounded blocks for the learned preconditioner (once
// per body set): every body of a type must share its body-frame blobs
int ensure_types(arb_ctx *ctx, hipStream_t s) {
    if (ctx->types_ready) return 0;
    const int M = ctx->M;
    int T = 0;
    for (int p = 0; p < M; ++p) T = std::max(T, ctx->h_body_type[p] + 1);
    std::vector<int> ref(T, -1);
    for (int p = 0; p < M; ++p) {
        const int t = ctx->h_body_type[p];
        if (t < 0) return fail(ctx, ARB_E_ARG, "negative body type");
        if (ref[t] < 0) {
            ref[t] = p;
            continue;
        }
        const int r = ref[t];
        const int nb = ctx->h_blob_off[p + 1] - ctx->h_blob_off[p];
        if (nb != ctx->h_blob_off[r + 1] - ctx->h_blob_off[r])
            return fail(ctx, ARB_E_ARG, "bodies of one type have different blob counts");
        for (int k = 0; k < 3 * nb; ++k)
            if (std::fabs(ctx->h_r_ref[3 * (size_t)ctx->h_blob_off[p] + k] -
                          ctx->h_r_ref[3 * (size_t)ctx->h_blob_off[r] + k]) > 1e-12)
                return fail(ctx, ARB_E_ARG, "bodies of one type have different body-frame blobs");
    }
    std::vector<int> tb(T + 1, 0);
    std::vector<double> pos;
    std::vector<int64_t> mo(T + 1, 0), zo(T + 1, 0);
    for (int t = 0; t < T; ++t) {
        const int r = ref[t];
        const int nb = r < 0 ? 0 : ctx->h_blob_off[r + 1] - ctx->h_blob_off[r];
        tb[t + 1] = tb[t] + nb;
        for (int k = 0; k < 3 * nb; ++k) pos.push_back(ctx->h_r_ref[3 * (size_t)ctx->h_blob_off[r] + k]);
        mo[t + 1] = mo[t] + 9 * (int64_t)nb * nb;
        zo[t + 1] = zo[t] + 18 * (int64_t)nb;
    }
    TRY(upload(ctx, ctx->t_blob_off, tb.data(), T + 1, s));
    TRY(upload(ctx, ctx->t_ref, pos.data(), pos.size(), s));
    TRY(upload(ctx, ctx->t_mat_off, mo.data(), T + 1, s));
    TRY(upload(ctx, ctx->t_z_off, zo.data(), T + 1, s));
    HIPCHK(ctx->t_mats.ensure(std::max<int64_t>(mo[T], 1) * sizeof(double)));
    HIPCHK(ctx->t_minv.ensure(std::max<int64_t>(mo[T], 1) * sizeof(double)));
    HIPCHK(ctx->t_Z.ensure(std::max<int64_t>(zo[T], 1) * sizeof(double)));
    HIPCHK(ctx->t_ldiag.ensure(std::max<size_t>(pos.size(), 1) * sizeof(double)));
    HIPCHK(ctx->t_dinv.ensure(arb::precond_dinv_size(tb[T], T) * sizeof(double)));
    HIPCHK(ctx->t_Nt.ensure(36 * (size_t)T * sizeof(double)));
    HIPCHK(ctx->t_body_pinv.ensure(std::max(T, 1) * sizeof(int)));
    HIPCHK(ctx->t_status.ensure(8 * sizeof(int)));
    HIPCHK(hipMemsetAsync(ctx->t_status.p, 0, 8 * sizeof(int), s));
    arb::PrecondDev P;
    P.M = T;
    P.blob_off = ctx->t_blob_off.as<int>();
    P.mat_off = ctx->t_mat_off.as<int64_t>();
    P.z_off = ctx->t_z_off.as<int64_t>();
    P.mats = ctx->t_mats.as<double>();
    P.minv = ctx->t_minv.as<double>();
    P.ldiag = ctx->t_ldiag.as<double>();
    P.dinv = ctx->t_dinv.as<double>();
    P.Z = ctx->t_Z.as<double>();
    P.Nt = ctx->t_Nt.as<double>();
    P.body_pinv = ctx->t_body_pinv.as<int>();
    P.status = ctx->t_status.as<int>();
    arb::precond_assemble(s, P, ctx->t_ref.as<double>(), ctx->opt.a, ctx->opt.eta, false);
    int t_max_m = 0;
    for (int t = 0; t < T; ++t) t_max_m = std::max(t_max_m, 3 * (tb[t + 1] - tb[t]));
    HIPCHK(arb::precond_factor(s, P, ctx->t_ref.as<double>(), t_max_m));
    int st[8];
    HIPCHK(hipMemcpyAsync(st, ctx->t_status.p, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[0]) return fail(ctx, ARB_E_NOT_SPD, "body-frame blob mobility of a type is not SPD");
    ctx->h_type_ref = ref;
    ctx->types_ready = true;
    return 0;
}

int mlp_ensure_ws(arb_ctx *ctx, int Bp) {
    HIPCHK(ctx->mlp_ws.ensure((size_t)arb::mlp_workspace_bytes(Bp)));
    return 0;
}

int precond_build_exact(arb_ctx *ctx, hipStream_t s);

// learned preconditioner build: network features -> N~_p; falls back to the
// exact build when a predicted factor is not a valid Cholesky factor
int precond_build_single(arb_ctx *ctx, hipStream_t s);

int precond_build(arb_ctx *ctx, hipStream_t s) {
    TRY(ready(ctx));
    ctx->pc_learned = false;
    ctx->pc_lcorr = false;
    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB) return precond_build_single(ctx, s);
    if (ctx->opt.precond == ARB_PC_BODYFRAME) {
        // free-space blocks of each body type, rotated: no per-solve factorisation
        TRY(ensure_types(ctx, s));
        const int M = ctx->M;
        HIPCHK(ctx->Nt.ensure(36 * (size_t)M * sizeof(double)));
        HIPCHK(ctx->pctmp.ensure(6 * (size_t)M * sizeof(double)));
        HIPCHK(ctx->status.ensure(8 * sizeof(int)));
        HIPCHK(hipMemsetAsync(ctx->status.p, 0, 8 * sizeof(int), s));
        arb::rotate_body_mobility(s, M, ctx->body_type_d.as<int>(), ctx->t_Nt.as<double>(),
                                  ctx->R9.as<double>(), ctx->Nt.as<double>());
        ctx->pc_learned = true;  // same per-type apply path
        arb::PrecondDev P = pc_view(ctx);
        HIPCHK(arb::precond_assembly(s, P));
        int st[8];
        HIPCHK(hipMemcpyAsync(st, ctx->status.p, sizeof(st), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ctx->pc_built = true;
        ctx->pc_pinv = st[1];
        return ctx->pc_pinv ? ARB_W_PINV_USED : ARB_OK;
    }
    if (ctx->opt.precond != ARB_PC_LEARNED) return precond_build_exact(ctx, s);
    if (!ctx->mlp_ready) return fail(ctx, ARB_E_ARG, "learned preconditioner without parameters");
    TRY(ensure_types(ctx, s));
    const int M = ctx->M;
    const int Bp = (M + 15) / 16 * 16;
    TRY(mlp_ensure_ws(ctx, Bp));
    HIPCHK(ctx->mlp_x.ensure((size_t)M * 7 * sizeof(float)));
    HIPCHK(ctx->Nt.ensure(36 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->pctmp.ensure(6 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->status.ensure(8 * sizeof(int)));
    HIPCHK(hipMemsetAsync(ctx->status.p, 0, 8 * sizeof(int), s));
    arb::mlp_features(s, M, ctx->q.as<double>(), ctx->theta.as<double>(), ctx->body_type_d.as<int>(),
                      ctx->opt.a, ctx->mlp_x.as<float>());
    float *Y = arb::mlp_forward(s, ctx->mlp_params.p, ctx->mlp_ws.p, M, Bp, ctx->mlp_x.as<float>());
    arb::mlp_mobility(s, ctx->mlp_params.p, M, Y, ctx->opt.a, ctx->opt.eta, ctx->Nt.as<double>(),
                      ctx->status.as<int>() + 4);
    HIPCHK(ctx->lcorr.ensure(108 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->stmp.ensure(6 * (size_t)M * sizeof(double)));
    arb::learned_correction(s, M, ctx->body_type_d.as<int>(), ctx->t_Nt.as<double>(),
                            ctx->R9.as<double>(), ctx->Nt.as<double>(), ctx->lcorr.as<double>(),
                            ctx->status.as<int>() + 4);
    ctx->pc_lcorr = true;
    arb::PrecondDev P = pc_view(ctx);
    HIPCHK(arb::precond_assembly(s, P));
    int st[8];
    HIPCHK(hipMemcpyAsync(st, ctx->status.p, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[4]) {
        ctx->pc_lcorr = false;
        const int rc = precond_build_exact(ctx, s);
        return rc < 0 ? rc : ARB_W_LEARNED_FALLBACK;
    }
    ctx->pc_learned = true;
    ctx->pc_built = true;
    ctx->pc_pinv = st[1];
    return ctx->pc_pinv ? ARB_W_PINV_USED : ARB_OK;
}

// single-blob bodies: N~_p = self blocks, G~_a = (C_a N~_a C_a^T)^-1 (Sec. 3.1)
int precond_build_single(arb_ctx *ctx, hipStream_t s) {
    const int M = ctx->M;
    HIPCHK(ctx->Nt.ensure(36 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->pctmp.ensure(6 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->status.ensure(8 * sizeof(int)));
    HIPCHK(hipMemsetAsync(ctx->status.p, 0, 8 * sizeof(int), s));
    TRY(ensure_zero_offsets(ctx, s));
    arb::single_blob_body_mobility(s, M, ctx->opt.a, ctx->opt.eta, ctx->Nt.as<double>());
    arb::PrecondDev P = pc_view(ctx);
    HIPCHK(arb::precond_assembly(s, P));
    int st[8];
    HIPCHK(hipMemcpyAsync(st, ctx->status.p, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->pc_built = true;
    ctx->pc_pinv = st[1];
    return ctx->pc_pinv ? ARB_W_PINV_USED : ARB_OK;
}

int precond_build_exact(arb_ctx *ctx, hipStream_t s) {
    TRY(ready(ctx));
    const int M = ctx->M;
    std::vector<int64_t> mo(M + 1, 0), zo(M + 1, 0);
    int max_m = 0;
    for (int p = 0; p < M; ++p) {
        const int64_t m = 3 * (int64_t)(ctx->h_blob_off[p + 1] - ctx->h_blob_off[p]);
        mo[p + 1] = mo[p] + m * m;
        zo[p + 1] = zo[p] + 6 * m;
        max_m = std::max(max_m, (int)m);
    }
    TRY(upload(ctx, ctx->mat_off, mo.data(), M + 1, s));
    TRY(upload(ctx, ctx->z_off, zo.data(), M + 1, s));
    HIPCHK(ctx->mats.ensure(std::max<int64_t>(mo[M], 1) * sizeof(double)));
    HIPCHK(ctx->minv.ensure(std::max<int64_t>(mo[M], 1) * sizeof(double)));
    HIPCHK(ctx->ldiag.ensure(3 * (size_t)ctx->N * sizeof(double)));
    HIPCHK(ctx->dinv.ensure(arb::precond_dinv_size(ctx->N, M) * sizeof(double)));
    HIPCHK(ctx->Z.ensure(std::max<int64_t>(zo[M], 1) * sizeof(double)));
    HIPCHK(ctx->Nt.ensure(36 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->body_pinv.ensure(std::max(M, 1) * sizeof(int)));
    HIPCHK(ctx->pctmp.ensure(6 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->status.ensure(8 * sizeof(int)));
    HIPCHK(hipMemsetAsync(ctx->status.p, 0, 8 * sizeof(int), s));
    arb::PrecondDev P = pc_view(ctx);
    arb::precond_assemble(s, P, ctx->pos.as<double>(), ctx->opt.a, ctx->opt.eta, ctx->opt.wall != 0);
    HIPCHK(arb::precond_factor(s, P, ctx->dvec.as<double>(), max_m));
    HIPCHK(arb::precond_assembly(s, P));
    int st[8];
    HIPCHK(hipMemcpyAsync(st, ctx->status.p, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[2]) return fail(ctx, ARB_E_BELOW_WALL, "a blob is at or below z = a with the wall on");
    if (st[0])
        return fail(ctx, ARB_E_NOT_SPD,
                    "blob mobility of body " + std::to_string(st[0] - 1) + " is not positive definite");
    ctx->pc_built = true;
    ctx->pc_pinv = st[1] + st[3];
    return ctx->pc_pinv ? ARB_W_PINV_USED : ARB_OK;
}

int precond_apply(arb_ctx *ctx, hipStream_t s, const double *r, double *z) {
    const int64_t n = n_unknowns(ctx);
    if (ctx->opt.precond == ARB_PC_NONE) {
        HIPCHK(hipMemcpyAsync(z, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        return 0;
    }
    arb::PrecondDev P = pc_view(ctx);
    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB)
        arb::precond_apply_single(s, P, ctx->zero_off.as<int>(), ctx->zero_off64.as<int64_t>(), r,
                                  z);
    else
        arb::precond_apply(s, P, ctx->N, r, z);
    return 0;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ---------------------------------------------------------------- GMRES (Sec. 3.1)
struct Krylov {
    int64_t n;
    int m, nch;
    double *b, *r, *z, *w, *V, *H, *cs, *sn, *g, *sv, *part, *h1, *h2, *sc;
    double *steps;  // gmres_small_cycle's per-step figures (2 m + 1)
};

int krylov_buffers(arb_ctx *ctx, Krylov &K) {
    const int64_t n = n_unknowns(ctx);
    const int m = ctx->opt.restart;
    K.n = n;
    K.m = m;
    K.nch = (int)((n + 2047) / 2048);
    HIPCHK(ctx->kb.ensure(n * sizeof(double)));
    HIPCHK(ctx->kr.ensure(n * sizeof(double)));
    HIPCHK(ctx->kz.ensure(n * sizeof(double)));
    HIPCHK(ctx->kw.ensure(n * sizeof(double)));
    HIPCHK(ctx->kt.ensure(2 * n * sizeof(double)));
    HIPCHK(ctx->kv.ensure((size_t)(m + 1) * n * sizeof(double)));
    HIPCHK(ctx->kH.ensure((size_t)(m + 1) * m * sizeof(double)));
    HIPCHK(ctx->kcs.ensure((size_t)(m + 1) * sizeof(double)));
    HIPCHK(ctx->ksn.ensure((size_t)(m + 1) * sizeof(double)));
    HIPCHK(ctx->kg.ensure((size_t)(m + 2) * sizeof(double)));
    HIPCHK(ctx->khcol.ensure((size_t)(2 * (m + 2) + 16) * sizeof(double)));
    HIPCHK(ctx->ksv.ensure((size_t)(m + 1) * sizeof(double)));
    HIPCHK(ctx->kpart.ensure((size_t)(m + 1) * K.nch * sizeof(double)));
    HIPCHK(ctx->ksteps.ensure((size_t)(2 * m + 2) * sizeof(double)));
    K.b = ctx->kb.as<double>();
    K.r = ctx->kr.as<double>();
    K.z = ctx->kz.as<double>();
    K.w = ctx->kw.as<double>();
    K.V = ctx->kv.as<double>();
    K.H = ctx->kH.as<double>();
    K.cs = ctx->kcs.as<double>();
    K.sn = ctx->ksn.as<double>();
    K.g = ctx->kg.as<double>();
    K.sv = ctx->ksv.as<double>();
    K.part = ctx->kpart.as<double>();
    K.h1 = ctx->khcol.as<double>();
    K.h2 = K.h1 + (m + 2);
    K.sc = K.h2 + (m + 2);  // 16 device scalars
    K.steps = ctx->ksteps.as<double>();
    return 0;
}

// Whether a GMRES cycle of this context runs in one workgroup (small.hip): a
// small multiblob FP64 system with the exact block preconditioner
arb::SmallSystem small_system(arb_ctx *ctx);

bool small_cycle_ok(arb_ctx *ctx, int prec, int64_t n) {
    return ctx->opt.small_cycle == 0 && ctx->opt.model == ARB_MODEL_MULTIBLOB &&
           prec == ARB_FP64 && ctx->opt.precond == ARB_PC_BLOCK && !ctx->pc_learned &&
           ctx->opt.pair_kernel != ARB_PAIR_FMM && !ctx->prof && ctx->M > 0 &&
           ctx->N <= arb::kSmallCycleN && n <= arb::kSmallArnoldi &&
           (ctx->n_asm == 0 || ctx->asm_max_rows <= arb::kSmallCycleRows) &&
           arb::small_layout(small_system(ctx)).bytes <= arb::kSmallCycleLds;
}

arb::SmallSystem small_system(arb_ctx *ctx) {
    const arb::PrecondDev P = pc_view(ctx);
    arb::SmallSystem S;
    S.N = ctx->N;
    S.M = ctx->M;
    S.Nc = ctx->Nc;
    S.A = ctx->n_asm;
    S.n = n_unknowns(ctx);
    S.wall = ctx->opt.wall != 0;
    S.a = ctx->opt.a;
    S.scale = 1.0 / (8.0 * arb::kPi * ctx->opt.eta);
    const bool so = ctx->psorted;
    S.p64 = (so ? ctx->p64s : ctx->p64).as<double4>();
    S.perm = so ? ctx->pperm.as<int>() : nullptr;
    S.bob = ctx->body_of_blob.as<int>();
    S.blob_off = ctx->blob_off.as<int>();
    S.dvec = ctx->dvec.as<double>();
    S.brow_ptr = ctx->brow_ptr.as<int>();
    S.brow_ent = ctx->brow_ent.as<int>();
    S.row_p = ctx->row_p.as<int>();
    S.row_q = ctx->row_q.as<int>();
    S.crow = ctx->crow.as<double>();
    S.mat_off = P.mat_off;
    S.z_off = P.z_off;
    S.minv = P.minv;
    S.Z = P.Z;
    S.Nt = P.Nt;
    S.asm_row_ptr = P.asm_row_ptr;
    S.asm_rows = P.asm_rows;
    S.asm_mat_off = P.asm_mat_off;
    S.G = P.G;
    for (int p = 0; p < S.M; ++p) {
        const int64_t mm = 3 * (int64_t)(ctx->h_blob_off[p + 1] - ctx->h_blob_off[p]);
        S.n_minv += mm * mm;
        S.n_z += 6 * mm;
    }
    for (int a = 0; a < S.A; ++a) {
        const int64_t na = ctx->h_asm_row_ptr[a + 1] - ctx->h_asm_row_ptr[a];
        S.n_g += na * na;
    }
    S.n_brow_ent = ctx->n_brow_ent;
    int tpt = 1;  // threads per target: the 512 threads in about one pass
    while (tpt < 64 && 2 * tpt * S.N <= 512) tpt *= 2;
    S.tpt = tpt;
    return S;
}

int dev_norm(arb_ctx *ctx, hipStream_t s, Krylov &K, const double *x, int slot, double *out) {
    arb::multidot(s, K.n, 1, x, K.n, x, K.part, K.sc + slot);
    HIPCHK(hipMemcpyAsync(ctx->pinned, K.sc + slot, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = std::sqrt(ctx->pinned[0]);
    return 0;
}

// Restarted GMRES on A P^-1 (right preconditioning) for A y = rhs, starting
// from the y already in place with its residual r = rhs - A y in K.r.  Stops
// when the residual of the operator in `prec` is <= tol_abs, or after the
// iteration budget.  Returns the final residual norm in *res (same operator).
// everything the launches of one Arnoldi step depend on besides buffer contents
std::vector<long long> graph_key(arb_ctx *ctx, const Krylov &K, int prec) {
    const int64_t skey = (int64_t)ctx->N * 4 + prec * 2 + (ctx->opt.wall ? 1 : 0);
    auto it = ctx->slice_cache.find(skey);
    return {(long long)arb::alloc_generation().load(), (long long)K.n, K.m, prec,
            ctx->opt.precond, ctx->opt.left_precond, ctx->psorted ? 1 : 0, ctx->pc_learned ? 1 : 0,
            ctx->pc_lcorr ? 1 : 0, ctx->N, ctx->M,
            ctx->Nc, ctx->n_asm, it == ctx->slice_cache.end() ? 0 : it->second,
            (long long)(intptr_t)K.V, (long long)(intptr_t)ctx->pinned, ctx->fmm.version};
}

// run one Arnoldi step: replay its graph, capturing it first if needed; plain
// launches if capture is unavailable
template <class F>
int run_step_graph(arb_ctx *ctx, hipStream_t s, int j, const std::vector<long long> &key,
                   F &&body) {
    GmresGraphs &G = ctx->ggraph;
    if (G.broken) return body();
    if (G.key != key) {
        G.clear();
        G.key = key;
    }
    if ((int)G.exec.size() <= j) G.exec.resize(j + 1, nullptr);
    if (!G.exec[j]) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            G.broken = true;
            return body();
        }
        const int rc = body();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        hipGraphExec_t x = nullptr;
        const hipError_t e2 =
            (rc == 0 && e == hipSuccess) ? hipGraphInstantiate(&x, g, nullptr, nullptr, 0) : e;
        if (g) (void)hipGraphDestroy(g);
        if (rc != 0 || e2 != hipSuccess) {
            // nothing recorded ran: fall back to plain launches for this context
            (void)hipGetLastError();
            if (x) (void)hipGraphExecDestroy(x);
            G.broken = true;
            return body();
        }
        G.exec[j] = x;
    }
    HIPCHK(hipGraphLaunch(G.exec[j], s));
    return 0;
}

// Restarted GMRES for A y = rhs (Sec. 3.1), starting from the y already in place
// with its residual r = rhs - A y in K.r.  Right preconditioning (A P^-1, the
// default): the Givens estimate is the residual of the operator in `prec`.
// Left preconditioning (opt.left_precond, P^-1 A from P^-1 r): the estimate is
// the preconditioned residual, and a cycle stops when it has fallen by the
// factor the true residual still has to fall.  Either way a cycle ends with
// the true residual recomputed (unless trust_estimate, for an inner solve
// whose caller recomputes it), and the loop stops when it is <= tol_abs or
// after the iteration budget.  Returns the final residual norm in *res.
//
// The host reads two scalars per Arnoldi step (h_{j+1,j} and the estimate) to
// decide when to stop.  When a step is cheap (at most 65,536 unknowns, or a first
// step under half a millisecond: steps that are launch-bound) the next step is
// enqueued before
// the host waits for the current one's scalars, so the device never idles on
// the host; a step launched past the stopping point only writes Krylov columns
// beyond those the update uses, so the result is the same.
int gmres_core(arb_ctx *ctx, hipStream_t s, Krylov &K, const double *rhs, double *y,
               double tol_abs, int prec, int max_iter, int *total, int *restarts,
               double hist_scale, arb_solve_info *inf, double *res, bool trust_estimate) {
    const int64_t n = K.n;
    const int m = K.m;
    const bool left = ctx->opt.left_precond != 0;
    double *pin = ctx->pinned;
    double *pin_step = ctx->pinned + kPinnedScalars;
    while ((int)ctx->step_ev.size() < m) {
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->step_ev.push_back(e);
    }
    auto push = [&](double v) {
        if (inf->history_len < 1024) inf->history[inf->history_len++] = v;
    };
    auto read_norm = [&](const double *x, int slot, double *out) -> int {
        arb::multidot(s, n, 1, x, n, x, K.part, K.sc + slot);
        arb::g_init(s, m, K.sc + slot, K.g, K.sc + 3);  // g = [norm, 0, ...], sc[3] = norm
        HIPCHK(hipMemcpyAsync(pin, K.sc + 3, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *out = pin[0];
        return 0;
    };
    // work counts (a replayed graph runs the same product and apply as step())
    auto count_product = [&]() { ++(prec == ARB_FP64 ? inf->products_fp64 : inf->products_fp32); };
    const bool graphs = ctx->opt.graphs == 0 && !ctx->prof;
    const bool small = n <= arb::kSmallArnoldi;
    // a whole cycle in one launch of one workgroup (stopping test on the device)
    const bool one_launch = !left && small_cycle_ok(ctx, prec, n);
    arb::SmallSystem SS;
    if (one_launch) SS = small_system(ctx);
    for (;;) {
        double beta = 0.0;
        TRY(read_norm(K.r, 2, &beta));
        if (!std::isfinite(beta)) return fail(ctx, ARB_E_NAN, "GMRES residual is not finite");
        *res = beta;
        push(beta * hist_scale);
        if (beta <= tol_abs || *total >= max_iter) break;
        double target = tol_abs, scale = 1.0;
        const double *start = K.r;
        if (left) {
            // Krylov space of P^-1 A from z0 = P^-1 r; g[0] = ||z0||
            TRY(precond_apply(ctx, s, K.r, K.z));
            ++inf->precond_applies;
            double bz = 0.0;
            TRY(read_norm(K.z, 2, &bz));
            if (!std::isfinite(bz) || bz == 0.0)
                return fail(ctx, ARB_E_NAN, "preconditioned residual is not finite or zero");
            target = tol_abs / beta * bz;
            scale = beta / bz;
            start = K.z;
        }
        arb::scale_copy(s, n, start, K.sc + 3, K.V);  // v_0 = start / ||start||
        // one Arnoldi step; the first of a cycle runs plainly (it may tune the
        // pair launch), the others replay a graph captured once per j
        auto step = [&](int j) -> int {
            double *vj = K.V + (size_t)j * n;
            if (j > 0) arb::scale_copy(s, n, K.w, K.sc + 5, vj);  // v_j = w / h_{j,j-1}
            if (left) {
                TRY(system_apply(ctx, s, vj, K.z, prec));
                TRY(precond_apply(ctx, s, K.z, K.w));
            } else {
                TRY(precond_apply(ctx, s, vj, K.z));
                TRY(system_apply(ctx, s, K.z, K.w, prec));
            }
            if (small) {
                arb::arnoldi_small(s, n, j, m, K.V, n, K.w, K.H, K.cs, K.sn, K.g, K.sc + 5);
            } else {
                // classical Gram-Schmidt, twice
                arb::multidot(s, n, j + 1, K.V, n, K.w, K.part, K.h1);
                arb::gemv_sub(s, n, j + 1, K.V, n, K.h1, K.w);
                arb::multidot(s, n, j + 1, K.V, n, K.w, K.part, K.h2);
                arb::gemv_sub(s, n, j + 1, K.V, n, K.h2, K.w);
                arb::multidot(s, n, 1, K.w, n, K.w, K.part, K.sc + 4);
                arb::arnoldi_post(s, j, m, K.h1, K.h2, K.sc + 4, K.H, K.cs, K.sn, K.g, K.sc + 5);
            }
            HIPCHK(hipMemcpyAsync(pin_step + 2 * j, K.sc + 5, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            return 0;
        };
        auto launch = [&](int j) -> int {
            if (graphs && j > 0) {
                const std::vector<long long> key = graph_key(ctx, K, prec);
                TRY(run_step_graph(ctx, s, j, key, [&]() { return step(j); }));
            } else {
                TRY(step(j));
            }
            HIPCHK(hipEventRecord(ctx->step_ev[j], s));
            return 0;
        };
        // steps may be launched up to `lag` ahead of the one the host checks; the
        // lag is chosen from the time of the cycle's first step
        int k = 0, launched = 0, lag = 0;
        const int budget = std::min(m, max_iter - *total);
        double last_est = beta;
        if (one_launch) {
            HIPCHK(arb::gmres_small_cycle(s, SS, m, budget, target, K.V, K.H, K.cs, K.sn, K.g,
                                          K.steps));
            HIPCHK(hipMemcpyAsync(pin_step, K.steps, (2 * (size_t)m + 1) * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            k = (int)pin_step[2 * m];
            if (k < 1 || k > budget) return fail(ctx, ARB_E_DEVICE, "GMRES cycle: bad step count");
            ++inf->one_launch_cycles;
            for (int j = 0; j < k; ++j) {
                const double est = pin_step[2 * j + 1];
                if (!std::isfinite(est))
                    return fail(ctx, ARB_E_NAN, "GMRES produced a non-finite value");
                ++*total;
                count_product();
                ++inf->precond_applies;
                push(est * scale * hist_scale);
                last_est = est;
            }
        }
        for (int j = 0; j < budget && !one_launch; ++j) {
            const double t_launch = now_ms();
            while (launched < budget && launched <= j + lag) TRY(launch(launched++));
            HIPCHK(hipEventSynchronize(ctx->step_ev[j]));
            if (j == 0) lag = (n <= 65536 || now_ms() - t_launch < 0.5) ? 1 : 0;
            const double hn = pin_step[2 * j], est = pin_step[2 * j + 1];
            if (!std::isfinite(est)) return fail(ctx, ARB_E_NAN, "GMRES produced a non-finite value");
            ++*total;
            count_product();
            ++inf->precond_applies;
            k = j + 1;
            push(est * scale * hist_scale);
            last_est = est;
            if (est <= target || hn == 0.0) break;
        }
        arb::upper_solve(s, k, m, K.H, K.g, K.sv);
        if (left) {
            arb::gemv_set(s, n, k, K.V, n, K.sv, K.z);
        } else {
            arb::gemv_set(s, n, k, K.V, n, K.sv, K.w);
            TRY(precond_apply(ctx, s, K.w, K.z));
            ++inf->precond_applies;
        }
        arb::axpby(s, n, 1.0, K.z, 1.0, y);
        ++*restarts;
        if (trust_estimate && last_est <= target) {
            // an outer loop recomputes the residual in higher precision
            *res = last_est * scale;
            return 0;
        }
        --*restarts;
        TRY(system_apply(ctx, s, y, K.r, prec));
        count_product();
        arb::axpby(s, n, 1.0, rhs, -1.0, K.r);  // r = rhs - A y
        ++*restarts;
        if (inf->history_len > 0) inf->history_len--;  // estimate replaced by the true residual
    }
    return 0;
}

int solve_dev(arb_ctx *ctx, const double *F, const double *us, double *y, int warm,
              arb_solve_info *info, hipStream_t s) {
    TRY(ready(ctx));
    if (us && ctx->opt.model == ARB_MODEL_SINGLE_BLOB)
        return fail(ctx, ARB_E_ARG, "single-blob model: no blob slip velocity");
    const int N = ctx->N, M = ctx->M, Nc = ctx->Nc;
    Krylov K;
    TRY(krylov_buffers(ctx, K));
    const int64_t n = K.n;
    const int prec = ctx->opt.precision;
    const double tol = ctx->opt.tol;
    arb_solve_info loc{};
    arb_solve_info *inf = info ? info : &loc;
    std::memset(inf, 0, sizeof(*inf));

    HIPCHK(hipStreamSynchronize(s));
    const double t0 = now_ms();
    int warn = 0;
    if (ctx->opt.precond != ARB_PC_NONE) {
        const int rc = precond_build(ctx, s);
        if (rc < 0) return rc;
        if (rc > 0) warn = rc;
        inf->pinv_used = ctx->pc_pinv;
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t1 = now_ms();
    inf->t_build_ms = t1 - t0;

    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB) {
        // b = [N F; B]
        TRY(body_mobility_dev(ctx, s, F, 1.0, nullptr, K.b, ARB_FP64));
        if (Nc > 0)
            HIPCHK(hipMemcpyAsync(K.b + 6 * (size_t)M, ctx->Bc.p, Nc * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
    } else {
        arb::rhs_assemble(s, N, M, Nc, us, F, ctx->Bc.as<double>(), K.b);
    }
    double bnorm = 0.0;
    TRY(dev_norm(ctx, s, K, K.b, 0, &bnorm));
    if (!std::isfinite(bnorm)) return fail(ctx, ARB_E_NAN, "right-hand side is not finite");
    if (bnorm == 0.0) {
        HIPCHK(hipMemsetAsync(y, 0, n * sizeof(double), s));
        HIPCHK(hipStreamSynchronize(s));
        inf->history[inf->history_len++] = 0.0;
        return ARB_OK;
    }
    if (warm) {
        TRY(system_apply(ctx, s, y, K.r, ARB_FP64));
        ++inf->products_fp64;
        arb::axpby(s, n, 1.0, K.b, -1.0, K.r);  // r = b - A y
    } else {
        HIPCHK(hipMemsetAsync(y, 0, n * sizeof(double), s));
        HIPCHK(hipMemcpyAsync(K.r, K.b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    int total = 0, restarts = 0;
    double res = 0.0;
    const int max_iter = ctx->opt.max_iter;
    if (prec == ARB_FP64) {
        TRY(gmres_core(ctx, s, K, K.b, y, tol * bnorm, ARB_FP64, max_iter, &total, &restarts,
                       1.0 / bnorm, inf, &res, false));
    } else {
        // GMRES iterative refinement: the correction equation A d = r is solved by
        // GMRES with the FP32 pair sum to a modest relative tolerance; r = b - A y
        // is formed with the FP64 pair sum, so the stopping test is FP64.  The
        // one exception is the last correction (unless refine_final = 1): once a
        // correction has been checked, the FP32 product's error on it is bounded
        // by rho = (||r_new|| + e) / ||r_old|| (e the inner GMRES residual, by the
        // triangle inequality), and a later correction whose inner residual plus
        // kRefineSafety rho ||r|| is within tol ||b|| is accepted on that bound
        // without a further FP64 product (right preconditioning only, where the
        // inner residual is the unpreconditioned one).
        double *rhs = ctx->kt.as<double>();     // current FP64 residual (inner rhs)
        double *d = rhs + n;                     // inner solution
        TRY(dev_norm(ctx, s, K, K.r, 1, &res));
        double rho = -1.0;  // no correction checked yet
        for (int outer = 0; outer < 30; ++outer) {
            inf->history[inf->history_len < 1024 ? inf->history_len++ : 1023] = res / bnorm;
            if (res <= tol * bnorm || total >= max_iter) break;
            HIPCHK(hipMemcpyAsync(rhs, K.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemsetAsync(d, 0, n * sizeof(double), s));
            const double eta = std::max(1e-4, 0.5 * tol * bnorm / res);
            double rin = 0.0;
            TRY(gmres_core(ctx, s, K, rhs, d, eta * res, ARB_FP32C, max_iter, &total, &restarts,
                           1.0 / bnorm, inf, &rin, true));
            arb::axpby(s, n, 1.0, d, 1.0, y);
            if (ctx->opt.refine_final == 0 && !ctx->opt.left_precond && rho >= 0.0 &&
                rin <= eta * res) {
                const double bound = rin + kRefineSafety * rho * res;
                if (bound <= tol * bnorm) {
                    res = bound;
                    inf->residual_bounded = 1;
                    inf->history[inf->history_len < 1024 ? inf->history_len++ : 1023] =
                        res / bnorm;
                    break;
                }
            }
            TRY(system_apply(ctx, s, y, K.r, ARB_FP64));
            ++inf->products_fp64;
            arb::axpby(s, n, 1.0, K.b, -1.0, K.r);
            const double res_old = res;
            TRY(dev_norm(ctx, s, K, K.r, 1, &res));
            if (!std::isfinite(res)) return fail(ctx, ARB_E_NAN, "refinement residual not finite");
            rho = (res + rin) / res_old;
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t2 = now_ms();
    inf->t_solve_ms = t2 - t1;
    inf->iterations = total;
    inf->restarts = restarts;
    inf->rel_residual = res / bnorm;
    inf->rel_residual_fp64 = res / bnorm;
    if (inf->rel_residual_fp64 > tol) return ARB_W_NOT_CONVERGED;
    return warn;
}

int check_finite(arb_ctx *ctx, const double *v, size_t n, const char *what) {
    if (!v) return 0;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return fail(ctx, ARB_E_NAN, std::string(what) + " is not finite");
    return 0;
}

// Entry points return ARB_E_HOST instead of letting a C++ exception (a failed
// host allocation, a thread that cannot start) cross the C ABI.
int guard_fail(const arb_ctx *c, const char *what) noexcept {
    try {
        if (c) const_cast<arb_ctx *>(c)->err = std::string("host failure: ") + what;
    } catch (...) {
    }
    return ARB_E_HOST;
}
#define ARB_GUARD_BEGIN try {
#define ARB_GUARD_END(c)                                           \
    }                                                              \
    catch (const std::bad_alloc &) {                               \
        return guard_fail(c, "host memory allocation failed");     \
    }                                                              \
    catch (const std::exception &e_) {                             \
        return guard_fail(c, e_.what());                           \
    }                                                              \
    catch (...) {                                                  \
        return guard_fail(c, "unknown exception");                 \
    }

}  // namespace

// ====================================================================== C ABI
extern "C" {

int arb_create(arb_ctx **out, const arb_options *opt) {
    ARB_GUARD_BEGIN
    arb_ctx *ctx = nullptr;
    if (!out || !opt) return ARB_E_ARG;
    *out = nullptr;
    if (!(opt->a > 0) || !(opt->eta > 0) || !(opt->tol > 0) || opt->restart < 1 ||
        opt->restart > arb::kMaxRestart || opt->max_iter < 1 ||
        (opt->precision != ARB_FP64 && opt->precision != ARB_FP32C) || opt->precond < 0 ||
        opt->precond > 3 || opt->slices < 0 || opt->slices > 4096 || opt->pair_kernel < 0 ||
        opt->pair_kernel > ARB_PAIR_FMM || opt->graphs < 0 || opt->graphs > 1 ||
        (opt->model != ARB_MODEL_MULTIBLOB && opt->model != ARB_MODEL_SINGLE_BLOB) ||
        (opt->fmm_order != 0 && (opt->fmm_order < 2 || opt->fmm_order > arb::kFmmMaxOrder)) ||
        opt->fmm_levels < 0 || opt->fmm_levels > arb::kFmmMaxLevel || opt->fmm_leaf < 0 ||
        opt->left_precond < 0 || opt->left_precond > 1 || opt->small_cycle < 0 ||
        opt->small_cycle > 1 || opt->refine_final < 0 || opt->refine_final > 1)
        return ARB_E_ARG;
    // single-blob bodies: unbounded generalised RPY, exact or no preconditioner,
    // direct sums
    if (opt->model == ARB_MODEL_SINGLE_BLOB && (opt->wall != 0 || opt->precond > ARB_PC_BLOCK))
        return ARB_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device < 0 || opt->device >= ndev)
        return ARB_E_DEVICE;
    if (hipSetDevice(opt->device) != hipSuccess) return ARB_E_DEVICE;
    // the allocation-free entry point's scratch address on this device (its
    // own calls report a failed lookup)
    (void)arb::noalloc_setup(opt->device);
    ctx = new arb_ctx();
    ctx->opt = *opt;
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&ctx->pinned, kPinnedTotal * sizeof(double),
                      hipHostMallocDefault) !=
            hipSuccess) {
        delete ctx;
        return ARB_E_DEVICE;
    }
    *out = ctx;
    return ARB_OK;
    ARB_GUARD_END(nullptr)
}

void arb_destroy(arb_ctx *ctx) {
    try {
    if (!ctx) return;
    (void)hipSetDevice(ctx->opt.device);
    (void)hipDeviceSynchronize();
    ctx->ggraph.clear();
    for (auto &e : ctx->prof_ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto &e : ctx->step_ev) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    } catch (...) {
    }
}

const char *arb_last_error(const arb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int arb_get_slices(const arb_ctx *ctx, int n_blobs) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (ctx->opt.slices > 0) return ctx->opt.slices;
    for (int prec = 0; prec < 2; ++prec) {
        const int64_t key = (int64_t)n_blobs * 4 + prec * 2 + (ctx->opt.wall ? 1 : 0);
        if (prec == ctx->opt.precision) {
            auto it = ctx->slice_cache.find(key);
            if (it != ctx->slice_cache.end()) return it->second;
        }
    }
    return heuristic_slices(n_blobs);
    ARB_GUARD_END(ctx)
}

int arb_set_bodies(arb_ctx *ctx, int M, const int32_t *blob_offset, const double *r_ref,
                   const int32_t *body_type) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (M <= 0 || !blob_offset || !r_ref) return fail(ctx, ARB_E_ARG, "bad body arguments");
    if (blob_offset[0] != 0) return fail(ctx, ARB_E_ARG, "blob_offset[0] must be 0");
    for (int p = 0; p < M; ++p) {
        const int nb = blob_offset[p + 1] - blob_offset[p];
        if (nb < 1) return fail(ctx, ARB_E_ARG, "every body needs at least one blob");
        if (nb > kMaxBodyBlobs) return fail(ctx, ARB_E_ARG, "more than 512 blobs in one body");
    }
    const int N = blob_offset[M];
    if (check_finite(ctx, r_ref, 3 * (size_t)N, "r_ref")) return ARB_E_NAN;
    if (ctx->opt.model == ARB_MODEL_SINGLE_BLOB) {
        if (N != M) return fail(ctx, ARB_E_ARG, "single-blob model: one blob per body");
        for (int i = 0; i < 3 * N; ++i)
            if (r_ref[i] != 0.0)
                return fail(ctx, ARB_E_ARG, "single-blob model: blobs sit at the tracking points");
    }
    HIPCHK(hipSetDevice(ctx->opt.device));
    ctx->M = M;
    ctx->N = N;
    ctx->h_blob_off.assign(blob_offset, blob_offset + M + 1);
    ctx->h_r_ref.assign(r_ref, r_ref + 3 * (size_t)N);
    ctx->h_body_of_blob.resize(N);
    for (int p = 0; p < M; ++p)
        for (int i = blob_offset[p]; i < blob_offset[p + 1]; ++i) ctx->h_body_of_blob[i] = p;
    if (body_type)
        ctx->h_body_type.assign(body_type, body_type + M);
    else
        ctx->h_body_type.assign(M, 0);
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->blob_off, ctx->h_blob_off.data(), M + 1, s));
    TRY(upload(ctx, ctx->body_of_blob, ctx->h_body_of_blob.data(), N, s));
    TRY(upload(ctx, ctx->r_ref, ctx->h_r_ref.data(), 3 * (size_t)N, s));
    TRY(upload(ctx, ctx->body_type_d, ctx->h_body_type.data(), M, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->types_ready = false;
    ctx->have_state = false;
    ctx->topo_dirty = true;
    ctx->lasm_dirty = true;
    ctx->pc_built = false;
    ctx->slice_cache.clear();
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_set_state(arb_ctx *ctx, const double *q, const double *theta) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (ctx->M <= 0) return fail(ctx, ARB_E_ARG, "bodies not set");
    if (!q || !theta) return fail(ctx, ARB_E_ARG, "null state");
    const int M = ctx->M;
    if (check_finite(ctx, q, 3 * (size_t)M, "q") || check_finite(ctx, theta, 4 * (size_t)M, "theta"))
        return ARB_E_NAN;
    for (int p = 0; p < M; ++p) {
        const double *t = theta + 4 * p;
        const double nn = t[0] * t[0] + t[1] * t[1] + t[2] * t[2] + t[3] * t[3];
        if (std::fabs(nn - 1.0) > 1e-8) return fail(ctx, ARB_E_ARG, "theta is not a unit quaternion");
    }
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->q, q, 3 * (size_t)M, s));
    TRY(upload(ctx, ctx->theta, theta, 4 * (size_t)M, s));
    TRY(build_topology(ctx));
    TRY(refresh_geometry(ctx, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->have_state = true;
    if (ctx->opt.wall) {
        HIPCHK(ctx->status.ensure(8 * sizeof(int)));
        int flag = arb::pair_wall_violation(s, ctx->N, ctx->p64.as<double4>(), ctx->opt.a,
                                            ctx->status.as<int>(), (int *)ctx->pinned);
        if (flag) return fail(ctx, ARB_E_BELOW_WALL, "a blob is at or below z = a with the wall on");
    }
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_blob_positions(arb_ctx *ctx, double *r_out) {
    ARB_GUARD_BEGIN
    if (!ctx || !r_out) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipMemcpyAsync(r_out, ctx->pos.p, 3 * (size_t)ctx->N * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_set_links(arb_ctx *ctx, int P, const int32_t *pq, const double *dl_p, const double *dl_q,
                  const double *dldot_p, const double *dldot_q, const int32_t *nproj,
                  const double *proj) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (P < 0 || (P > 0 && (!pq || !dl_p || !dl_q))) return fail(ctx, ARB_E_ARG, "bad link arguments");
    ctx->P = P;
    ctx->h_pq.assign(pq, pq + 2 * (size_t)P);
    ctx->h_dl_p.assign(dl_p, dl_p + 3 * (size_t)P);
    ctx->h_dl_q.assign(dl_q, dl_q + 3 * (size_t)P);
    ctx->h_dldot_p.assign(3 * (size_t)P, 0.0);
    ctx->h_dldot_q.assign(3 * (size_t)P, 0.0);
    if (dldot_p) ctx->h_dldot_p.assign(dldot_p, dldot_p + 3 * (size_t)P);
    if (dldot_q) ctx->h_dldot_q.assign(dldot_q, dldot_q + 3 * (size_t)P);
    ctx->h_nproj.assign(P, 3);
    ctx->h_proj.assign(9 * (size_t)P, 0.0);
    for (int n = 0; n < P; ++n) {
        if (nproj) {
            if (nproj[n] < 1 || nproj[n] > 3) return fail(ctx, ARB_E_ARG, "nproj must be 1..3");
            ctx->h_nproj[n] = nproj[n];
        }
        for (int k = 0; k < 9; ++k)
            ctx->h_proj[9 * n + k] = proj ? proj[9 * n + k] : ((k % 4 == 0) ? 1.0 : 0.0);
    }
    if (check_finite(ctx, ctx->h_dl_p.data(), ctx->h_dl_p.size(), "dl_p") ||
        check_finite(ctx, ctx->h_dl_q.data(), ctx->h_dl_q.size(), "dl_q") ||
        check_finite(ctx, ctx->h_proj.data(), ctx->h_proj.size(), "proj"))
        return ARB_E_NAN;
    ctx->topo_dirty = true;
    ctx->lasm_dirty = true;
    ctx->pc_built = false;
    if (ctx->have_state) {
        HIPCHK(hipSetDevice(ctx->opt.device));
        TRY(build_topology(ctx));
        TRY(refresh_rows(ctx, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_set_rows(arb_ctx *ctx, int R, const int32_t *pq, const double *coef, const double *rhs) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (R < 0 || (R > 0 && (!pq || !coef || !rhs))) return fail(ctx, ARB_E_ARG, "bad row arguments");
    ctx->Rg = R;
    ctx->h_gpq.assign(pq, pq + 2 * (size_t)R);
    ctx->h_gcoef.assign(coef, coef + 12 * (size_t)R);
    ctx->h_grhs.assign(rhs, rhs + (size_t)R);
    if (check_finite(ctx, ctx->h_gcoef.data(), ctx->h_gcoef.size(), "coef") ||
        check_finite(ctx, ctx->h_grhs.data(), ctx->h_grhs.size(), "rhs"))
        return ARB_E_NAN;
    ctx->topo_dirty = true;
    ctx->lasm_dirty = true;
    ctx->pc_built = false;
    if (ctx->have_state) {
        HIPCHK(hipSetDevice(ctx->opt.device));
        TRY(build_topology(ctx));
        TRY(refresh_rows(ctx, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_sizes(const arb_ctx *ctx, int *N, int *M, int *Nc, int64_t *n) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    int nc = ctx->Nc;
    if (ctx->topo_dirty) {
        nc = ctx->Rg;
        for (int k : ctx->h_nproj) nc += k;
    }
    if (N) *N = ctx->N;
    if (M) *M = ctx->M;
    if (Nc) *Nc = nc;
    if (n)
        *n = (ctx->opt.model == ARB_MODEL_SINGLE_BLOB ? 0 : 3 * (int64_t)ctx->N) +
             6 * (int64_t)ctx->M + nc;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_fmm_get_stats(const arb_ctx *ctx, arb_fmm_stats *out) {
    ARB_GUARD_BEGIN
    if (!ctx || !out) return ARB_E_ARG;
    const arb::FmmState &F = ctx->fmm;
    if (ctx->opt.pair_kernel != ARB_PAIR_FMM || !F.ready) return ARB_E_ARG;
    out->levels = F.L;
    out->order = F.n;
    out->cells = F.ncell;
    out->leaves = F.nleaf;
    out->near_pairs = F.n_near_pairs;
    out->interactions = F.n_il;
    out->m2l_pairs = F.n_m2l_pairs;
    out->build_ms = F.build_ms;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mobility_apply_dev(arb_ctx *ctx, const double *lambda_dev, double *u_dev, void *stream) {
    ARB_GUARD_BEGIN
    if (!ctx || !lambda_dev || !u_dev) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    TRY(ctx_pair(ctx, pick(ctx, stream), lambda_dev, u_dev, nullptr, ctx->opt.precision));
    HIPCHK(hipGetLastError());
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mobility_apply(arb_ctx *ctx, const double *lambda, double *u) {
    ARB_GUARD_BEGIN
    if (!ctx || !lambda || !u) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    const size_t n3 = 3 * (size_t)ctx->N;
    if (check_finite(ctx, lambda, n3, "lambda")) return ARB_E_NAN;
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, lambda, n3, s));
    HIPCHK(ctx->s_out.ensure(n3 * sizeof(double)));
    TRY(ctx_pair(ctx, s, ctx->s_in.as<double>(), ctx->s_out.as<double>(), nullptr,
                 ctx->opt.precision));
    HIPCHK(hipMemcpyAsync(u, ctx->s_out.p, n3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_rpy_apply_dev(arb_ctx *ctx, int N, const double *pos_dev, const double *lambda_dev,
                      double *u_dev, void *stream) {
    ARB_GUARD_BEGIN
    if (!ctx || N < 0 || (N > 0 && (!pos_dev || !lambda_dev || !u_dev))) return ARB_E_ARG;
    if (N == 0) return ARB_OK;
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = pick(ctx, stream);
    const size_t ntb = 2 * (size_t)((N + 63) / 64);
    HIPCHK(ctx->s_pos.ensure((size_t)N * (sizeof(double4) + 2 * sizeof(float4)) +
                             ntb * sizeof(float4)));
    double4 *p64 = ctx->s_pos.as<double4>();
    float4 *hi = reinterpret_cast<float4 *>(p64 + N);
    float4 *lo = hi + N;
    float4 *box = lo + N;
    arb::prep_positions(s, N, pos_dev, ctx->opt.a, p64, hi, lo, box, nullptr);
    if (ctx->opt.pair_kernel == ARB_PAIR_FMM) {
        // a tree of these positions; the context's own is rebuilt at its next product
        TRY(fmm_pair(ctx, s, N, pos_dev, hi, lo, lambda_dev, u_dev, nullptr, nullptr, nullptr,
                     true, ctx->opt.precision));
        ctx->fmm.dirty = true;
        HIPCHK(hipGetLastError());
        return ARB_OK;
    }
    const bool wall = ctx->opt.wall != 0;
    int sl = 0;
    TRY(choose_slices(ctx, s, N, p64, hi, lo, box, nullptr, lambda_dev, ctx->opt.precision, wall,
                      &sl));
    TRY(run_pair(ctx, s, N, p64, hi, lo, box, nullptr, lambda_dev, u_dev, nullptr, nullptr, nullptr,
                 ctx->opt.precision, wall, sl));
    HIPCHK(hipGetLastError());
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_rpy_apply(arb_ctx *ctx, int N, const double *pos, const double *lambda, double *u) {
    ARB_GUARD_BEGIN
    if (!ctx || N < 0 || (N > 0 && (!pos || !lambda || !u))) return ARB_E_ARG;
    if (N == 0) return ARB_OK;
    if (check_finite(ctx, pos, 3 * (size_t)N, "pos") ||
        check_finite(ctx, lambda, 3 * (size_t)N, "lambda"))
        return ARB_E_NAN;
    if (ctx->opt.wall)
        for (int i = 0; i < N; ++i)
            if (!(pos[3 * i + 2] > ctx->opt.a))
                return fail(ctx, ARB_E_BELOW_WALL, "a blob is at or below z = a with the wall on");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    const size_t n3 = 3 * (size_t)N;
    TRY(upload(ctx, ctx->s_in, pos, n3, s));
    TRY(upload(ctx, ctx->s_aux, lambda, n3, s));
    HIPCHK(ctx->s_out.ensure(n3 * sizeof(double)));
    TRY(arb_rpy_apply_dev(ctx, N, ctx->s_in.as<double>(), ctx->s_aux.as<double>(),
                          ctx->s_out.as<double>(), s));
    HIPCHK(hipMemcpyAsync(u, ctx->s_out.p, n3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_body_mobility_apply_dev(arb_ctx *ctx, const double *FT_dev, double *UW_dev,
                                void *stream) {
    ARB_GUARD_BEGIN
    if (!ctx || !FT_dev || !UW_dev) return ARB_E_ARG;
    if (ctx->opt.model != ARB_MODEL_SINGLE_BLOB)
        return fail(ctx, ARB_E_ARG, "body mobility product needs the single-blob model");
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    TRY(body_mobility_dev(ctx, s, FT_dev, 1.0, nullptr, UW_dev, ctx->opt.precision));
    HIPCHK(hipGetLastError());
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_body_mobility_apply(arb_ctx *ctx, const double *FT, double *UW) {
    ARB_GUARD_BEGIN
    if (!ctx || !FT || !UW) return ARB_E_ARG;
    if (ctx->opt.model != ARB_MODEL_SINGLE_BLOB)
        return fail(ctx, ARB_E_ARG, "body mobility product needs the single-blob model");
    TRY(ready(ctx));
    const size_t m6 = 6 * (size_t)ctx->M;
    if (check_finite(ctx, FT, m6, "FT")) return ARB_E_NAN;
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, FT, m6, s));
    HIPCHK(ctx->s_out.ensure(m6 * sizeof(double)));
    TRY(body_mobility_dev(ctx, s, ctx->s_in.as<double>(), 1.0, nullptr, ctx->s_out.as<double>(),
                          ctx->opt.precision));
    HIPCHK(hipMemcpyAsync(UW, ctx->s_out.p, m6 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_system_apply(arb_ctx *ctx, const double *y, double *out) {
    ARB_GUARD_BEGIN
    if (!ctx || !y || !out) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    const int64_t n = n_unknowns(ctx);
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, y, n, s));
    HIPCHK(ctx->s_out.ensure(n * sizeof(double)));
    TRY(system_apply(ctx, s, ctx->s_in.as<double>(), ctx->s_out.as<double>(), ctx->opt.precision));
    HIPCHK(hipMemcpyAsync(out, ctx->s_out.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_K_apply(arb_ctx *ctx, const double *U, double *out) {
    ARB_GUARD_BEGIN
    if (!ctx || !U || !out) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, U, 6 * (size_t)ctx->M, s));
    HIPCHK(ctx->s_out.ensure(3 * (size_t)ctx->N * sizeof(double)));
    arb::K_apply(s, ctx->N, ctx->body_of_blob.as<int>(), ctx->dvec.as<double>(),
                 ctx->s_in.as<double>(), ctx->s_out.as<double>());
    HIPCHK(hipMemcpyAsync(out, ctx->s_out.p, 3 * (size_t)ctx->N * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_KT_apply(arb_ctx *ctx, const double *lambda, double *out) {
    ARB_GUARD_BEGIN
    if (!ctx || !lambda || !out) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, lambda, 3 * (size_t)ctx->N, s));
    HIPCHK(ctx->s_out.ensure(6 * (size_t)ctx->M * sizeof(double)));
    arb::KT_CT_apply(s, ctx->M, ctx->blob_off.as<int>(), ctx->dvec.as<double>(),
                     ctx->s_in.as<double>(), 1.0, nullptr, nullptr, nullptr, nullptr,
                     ctx->s_out.as<double>());
    HIPCHK(hipMemcpyAsync(out, ctx->s_out.p, 6 * (size_t)ctx->M * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_constraint_rows(arb_ctx *ctx, double *coef, int32_t *pq, double *B) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    const int Nc = ctx->Nc;
    if (Nc == 0) return ARB_OK;
    if (coef)
        HIPCHK(hipMemcpyAsync(coef, ctx->crow.p, 12 * (size_t)Nc * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    if (B) HIPCHK(hipMemcpyAsync(B, ctx->Bc.p, (size_t)Nc * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<int> rp(Nc), rq(Nc);
    HIPCHK(hipMemcpyAsync(rp.data(), ctx->row_p.p, Nc * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rq.data(), ctx->row_q.p, Nc * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (pq)
        for (int k = 0; k < Nc; ++k) {
            pq[2 * k] = rp[k];
            pq[2 * k + 1] = rq[k];
        }
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_precond_build(arb_ctx *ctx) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    HIPCHK(hipSetDevice(ctx->opt.device));
    return precond_build(ctx, ctx->stream);
    ARB_GUARD_END(ctx)
}

int arb_precond_apply(arb_ctx *ctx, const double *r, double *z) {
    ARB_GUARD_BEGIN
    if (!ctx || !r || !z) return ARB_E_ARG;
    TRY(ready(ctx));
    if (ctx->opt.precond != ARB_PC_NONE && !ctx->pc_built)
        return fail(ctx, ARB_E_ARG, "preconditioner not built for the current state");
    HIPCHK(hipSetDevice(ctx->opt.device));
    const int64_t n = n_unknowns(ctx);
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, r, n, s));
    HIPCHK(ctx->s_out.ensure(n * sizeof(double)));
    TRY(precond_apply(ctx, s, ctx->s_in.as<double>(), ctx->s_out.as<double>()));
    HIPCHK(hipMemcpyAsync(z, ctx->s_out.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_precond_block(arb_ctx *ctx, int p, double *L, double *Ntilde) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    if (!ctx->pc_built) return fail(ctx, ARB_E_ARG, "preconditioner not built");
    if (p < 0 || p >= ctx->M) return fail(ctx, ARB_E_ARG, "body index out of range");
    if (L && ctx->pc_learned)
        return fail(ctx, ARB_E_ARG, "the per-type preconditioners have no per-body factor");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    int64_t off = 0;
    for (int k = 0; k < p; ++k) {
        const int64_t m = 3 * (int64_t)(ctx->h_blob_off[k + 1] - ctx->h_blob_off[k]);
        off += m * m;
    }
    const int64_t m = 3 * (int64_t)(ctx->h_blob_off[p + 1] - ctx->h_blob_off[p]);
    int max_m = 0;
    for (int k = 0; k < ctx->M; ++k)
        max_m = std::max(max_m, 3 * (ctx->h_blob_off[k + 1] - ctx->h_blob_off[k]));
    if (L) {
        HIPCHK(hipMemcpyAsync(L, ctx->mats.as<double>() + off, m * m * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    }
    if (Ntilde)
        HIPCHK(hipMemcpyAsync(Ntilde, ctx->Nt.as<double>() + 36 * (size_t)p, 36 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (L) {
        // the inverse was formed out of place: factor the kept block here
        if (!arb::precond_factor_in_place(max_m) && host_cholesky(L, (int)m) != 0)
            return fail(ctx, ARB_E_NOT_SPD, "blob mobility block is not positive definite");
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = i + 1; j < m; ++j) L[i * m + j] = 0.0;
    }
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_solve_dev(arb_ctx *ctx, const double *F_dev, const double *u_slip_dev, double *y_dev,
                  int warm, arb_solve_info *info, void *stream) {
    ARB_GUARD_BEGIN
    if (!ctx || !F_dev || !y_dev) return ARB_E_ARG;
    HIPCHK(hipSetDevice(ctx->opt.device));
    return solve_dev(ctx, F_dev, u_slip_dev, y_dev, warm, info, pick(ctx, stream));
    ARB_GUARD_END(ctx)
}

int arb_solve(arb_ctx *ctx, const double *F, const double *u_slip, const double *y0, double *U,
              double *phi, double *lambda, arb_solve_info *info) {
    ARB_GUARD_BEGIN
    if (!ctx || !F) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    const int N = ctx->N, M = ctx->M;
    const int64_t n = n_unknowns(ctx);
    if (check_finite(ctx, F, 6 * (size_t)M, "F") ||
        check_finite(ctx, u_slip, u_slip ? 3 * (size_t)N : 0, "u_slip") ||
        check_finite(ctx, y0, y0 ? (size_t)n : 0, "y0"))
        return ARB_E_NAN;
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, F, 6 * (size_t)M, s));
    if (u_slip) TRY(upload(ctx, ctx->s_aux, u_slip, 3 * (size_t)N, s));
    HIPCHK(ctx->ky.ensure(n * sizeof(double)));
    if (y0) HIPCHK(hipMemcpyAsync(ctx->ky.p, y0, n * sizeof(double), hipMemcpyHostToDevice, s));
    const int rc = solve_dev(ctx, ctx->s_in.as<double>(), u_slip ? ctx->s_aux.as<double>() : nullptr,
                             ctx->ky.as<double>(), y0 ? 1 : 0, info, s);
    if (rc < 0) return rc;
    ctx->ky_n = n;
    const double *yd = ctx->ky.as<double>();
    const int64_t uo = u_offset(ctx);
    if (lambda && ctx->opt.model != ARB_MODEL_SINGLE_BLOB)
        HIPCHK(hipMemcpyAsync(lambda, yd, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (U)
        HIPCHK(hipMemcpyAsync(U, yd + uo, 6 * (size_t)M * sizeof(double), hipMemcpyDeviceToHost,
                              s));
    if (phi && ctx->Nc > 0)
        HIPCHK(hipMemcpyAsync(phi, yd + uo + 6 * (size_t)M, ctx->Nc * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return rc;
    ARB_GUARD_END(ctx)
}

int arb_euler_update(arb_ctx *ctx, const double *U, double dt, double *q, double *theta) {
    ARB_GUARD_BEGIN
    if (!ctx || !U) return ARB_E_ARG;
    TRY(ready(ctx));
    if (check_finite(ctx, U, 6 * (size_t)ctx->M, "U")) return ARB_E_NAN;
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->s_in, U, 6 * (size_t)ctx->M, s));
    arb::euler_update(s, ctx->M, ctx->s_in.as<double>(), dt, ctx->q.as<double>(),
                      ctx->theta.as<double>());
    TRY(refresh_geometry(ctx, s));
    if (q)
        HIPCHK(hipMemcpyAsync(q, ctx->q.p, 3 * (size_t)ctx->M * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    if (theta)
        HIPCHK(hipMemcpyAsync(theta, ctx->theta.p, 4 * (size_t)ctx->M * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

// Articulated bodies of the link graph (bodies joined by links; bodies without
// links are left out) with their bodies and links, the correction's workspace
// offsets, and for the reconstruction each body's signed link list and
// G = (L + 1 1^T / M_a)^-1 (L^-1 with a link to a lab point), L = Phat^T Phat
// the body graph's Laplacian.  Rebuilt when bodies or links change.
static int link_assemblies(arb_ctx *ctx, hipStream_t s) {
    if (!ctx->lasm_dirty) return 0;
    const int M = ctx->M, P = ctx->P;
    std::vector<int> parent(M);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int i) {
        while (parent[i] != i) {
            parent[i] = parent[parent[i]];
            i = parent[i];
        }
        return i;
    };
    for (int n = 0; n < P; ++n) {
        const int p = ctx->h_pq[2 * n], qq = ctx->h_pq[2 * n + 1];
        if (qq >= 0) {
            const int a = find(p), b = find(qq);
            if (a != b) parent[std::max(a, b)] = std::min(a, b);
        }
    }
    std::vector<int> label(M, -1), has_link(M, 0);
    for (int n = 0; n < P; ++n) {
        has_link[ctx->h_pq[2 * n]] = 1;
        if (ctx->h_pq[2 * n + 1] >= 0) has_link[ctx->h_pq[2 * n + 1]] = 1;
    }
    int A = 0;
    std::vector<int> root_label(M, -1);
    for (int p = 0; p < M; ++p) {
        if (!has_link[p]) continue;
        const int r = find(p);
        if (root_label[r] < 0) root_label[r] = A++;
        label[p] = root_label[r];
    }
    ctx->lasm_A = A;
    ctx->lasm_fits_corr = true;
    if (A == 0) {
        ctx->lasm_dirty = false;
        return 0;
    }
    std::vector<int> abp(A + 1, 0), ab, alp(A + 1, 0), al(P), loc(M, -1);
    for (int p = 0; p < M; ++p)
        if (label[p] >= 0) abp[label[p] + 1]++;
    for (int a = 0; a < A; ++a) abp[a + 1] += abp[a];
    ab.assign(abp[A], 0);
    {
        std::vector<int> f2(abp.begin(), abp.end() - 1);
        for (int p = 0; p < M; ++p)
            if (label[p] >= 0) {
                loc[p] = f2[label[p]] - abp[label[p]];
                ab[f2[label[p]]++] = p;
            }
    }
    for (int n = 0; n < P; ++n) alp[label[ctx->h_pq[2 * n]] + 1]++;
    for (int a = 0; a < A; ++a) alp[a + 1] += alp[a];
    {
        std::vector<int> f2(alp.begin(), alp.end() - 1);
        for (int n = 0; n < P; ++n) al[f2[label[ctx->h_pq[2 * n]]]++] = n;
    }
    // correction workspace
    std::vector<int64_t> wo(A + 1, 0);
    for (int a = 0; a < A; ++a) {
        const int nb = abp[a + 1] - abp[a], nl = alp[a + 1] - alp[a];
        if (3 * nl + nb > kMaxCorrRows) ctx->lasm_fits_corr = false;
        wo[a + 1] = wo[a] + (ctx->lasm_fits_corr ? arb::correct_ws_doubles(nb, nl) : 0);
    }
    ctx->lasm_ws = ctx->lasm_fits_corr ? wo[A] : 0;
    // reconstruction: signed link lists per body, anchored flags, G per articulated body
    std::vector<int> adj_ptr(abp[A] + 1, 0), adj, anch(A, 0);
    std::vector<int64_t> goff(A + 1, 0);
    for (int a = 0; a < A; ++a) {
        const int nb = abp[a + 1] - abp[a];
        if (nb > kMaxReconBodies)
            return fail(ctx, ARB_E_ARG, "articulated body has more bodies than the reconstruction takes");
        goff[a + 1] = goff[a] + (int64_t)nb * nb;
        for (int e = 0; e < alp[a + 1] - alp[a]; ++e) {
            const int n = al[alp[a] + e];
            adj_ptr[abp[a] + loc[ctx->h_pq[2 * n]] + 1]++;
            if (ctx->h_pq[2 * n + 1] >= 0)
                adj_ptr[abp[a] + loc[ctx->h_pq[2 * n + 1]] + 1]++;
            else
                anch[a] = 1;
        }
    }
    for (int k = 0; k < abp[A]; ++k) adj_ptr[k + 1] += adj_ptr[k];
    adj.assign(adj_ptr[abp[A]], 0);
    std::vector<double> G(goff[A], 0.0);
    {
        std::vector<int> f2(adj_ptr.begin(), adj_ptr.end() - 1);
        for (int a = 0; a < A; ++a) {
            const int nb = abp[a + 1] - abp[a];
            double *La = G.data() + goff[a];
            for (int e = 0; e < alp[a + 1] - alp[a]; ++e) {
                const int n = al[alp[a] + e];
                const int lp = loc[ctx->h_pq[2 * n]], qq = ctx->h_pq[2 * n + 1];
                adj[f2[abp[a] + lp]++] = 2 * e;
                La[(size_t)lp * nb + lp] += 1.0;
                if (qq >= 0) {
                    const int lq = loc[qq];
                    adj[f2[abp[a] + lq]++] = 2 * e + 1;
                    La[(size_t)lq * nb + lq] += 1.0;
                    La[(size_t)lp * nb + lq] -= 1.0;
                    La[(size_t)lq * nb + lp] -= 1.0;
                }
            }
            if (!anch[a])
                for (int64_t k = 0; k < (int64_t)nb * nb; ++k) La[k] += 1.0 / nb;
            if (spd_inverse(La, nb) != 0)
                return fail(ctx, ARB_E_ARG, "link graph of an articulated body is singular");
        }
    }
    TRY(upload(ctx, ctx->c_link_ptr, alp.data(), A + 1, s));
    TRY(upload(ctx, ctx->c_links, al.data(), P, s));
    TRY(upload(ctx, ctx->c_local, loc.data(), M, s));
    TRY(upload(ctx, ctx->c_ws_off, wo.data(), A + 1, s));
    TRY(upload(ctx, ctx->c_pq, ctx->h_pq.data(), 2 * (size_t)P, s));
    TRY(upload(ctx, ctx->c_abp, abp.data(), A + 1, s));
    TRY(upload(ctx, ctx->c_ab, ab.data(), ab.size(), s));
    TRY(upload(ctx, ctx->r_adj_ptr, adj_ptr.data(), adj_ptr.size(), s));
    TRY(upload(ctx, ctx->r_adj, adj.data(), std::max<size_t>(adj.size(), 1), s));
    TRY(upload(ctx, ctx->r_anch, anch.data(), A, s));
    TRY(upload(ctx, ctx->r_goff, goff.data(), A + 1, s));
    TRY(upload(ctx, ctx->r_G, G.data(), G.size(), s));
    HIPCHK(ctx->c_ws.ensure(std::max<int64_t>(ctx->lasm_ws, 1) * sizeof(double)));
    HIPCHK(ctx->c_iters.ensure(A * sizeof(int)));
    HIPCHK(ctx->c_resid.ensure(A * sizeof(double)));
    HIPCHK(ctx->r_z.ensure(std::max<int64_t>(3 * (int64_t)P, 1) * sizeof(double)));
    HIPCHK(ctx->r_b.ensure(std::max<int64_t>(3 * (int64_t)abp[A], 1) * sizeof(double)));
    HIPCHK(ctx->r_ginf.ensure(A * sizeof(double)));
    HIPCHK(ctx->r_g2.ensure(A * sizeof(double)));
    HIPCHK(hipStreamSynchronize(s));  // the host vectors above end with this scope
    ctx->lasm_dirty = false;
    return 0;
}

// correction of every articulated body on stream s (state on the device)
static int correct_run(arb_ctx *ctx, hipStream_t s, double tol, int max_iter, int *iters,
                       double *resid) {
    TRY(link_assemblies(ctx, s));
    const int A = ctx->lasm_A;
    if (iters) *iters = 0;
    if (resid) *resid = 0.0;
    if (A == 0) return 0;
    if (!ctx->lasm_fits_corr)
        return fail(ctx, ARB_E_ARG, "articulated body too large for the correction kernel");
    arb::CorrectDev C;
    C.A = A;
    C.M = ctx->M;
    C.P = ctx->P;
    C.asm_body_ptr = ctx->c_abp.as<int>();
    C.asm_bodies = ctx->c_ab.as<int>();
    C.asm_link_ptr = ctx->c_link_ptr.as<int>();
    C.asm_links = ctx->c_links.as<int>();
    C.local_index = ctx->c_local.as<int>();
    C.pq = ctx->c_pq.as<int>();
    C.dl_p = ctx->dl_p.as<double>();
    C.dl_q = ctx->dl_q.as<double>();
    C.ws_off = ctx->c_ws_off.as<int64_t>();
    C.ws = ctx->c_ws.as<double>();
    C.q = ctx->q.as<double>();
    C.theta = ctx->theta.as<double>();
    C.iters = ctx->c_iters.as<int>();
    C.resid = ctx->c_resid.as<double>();
    arb::correct_positions(s, C, tol, max_iter);
    HIPCHK(hipGetLastError());
    std::vector<int> it(A);
    std::vector<double> rs(A);
    HIPCHK(hipMemcpyAsync(it.data(), C.iters, A * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rs.data(), C.resid, A * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (iters) *iters = *std::max_element(it.begin(), it.end());
    if (resid) *resid = *std::max_element(rs.begin(), rs.end());
    return 0;
}

// reconstruction (rebuild != 0) and/or link residual on stream s: g_inf = the
// largest |g_n component|, g2 = sum of g_n . g_n over all links
static int recon_run(arb_ctx *ctx, hipStream_t s, int rebuild, double *g_inf, double *g2) {
    TRY(link_assemblies(ctx, s));
    const int A = ctx->lasm_A;
    *g_inf = 0.0;
    *g2 = 0.0;
    if (A == 0) return 0;
    arb::ReconDev D;
    D.A = A;
    D.asm_body_ptr = ctx->c_abp.as<int>();
    D.asm_bodies = ctx->c_ab.as<int>();
    D.asm_link_ptr = ctx->c_link_ptr.as<int>();
    D.asm_links = ctx->c_links.as<int>();
    D.adj_ptr = ctx->r_adj_ptr.as<int>();
    D.adj = ctx->r_adj.as<int>();
    D.pq = ctx->c_pq.as<int>();
    D.anchored = ctx->r_anch.as<int>();
    D.g_off = ctx->r_goff.as<int64_t>();
    D.G = ctx->r_G.as<double>();
    D.dl_p = ctx->dl_p.as<double>();
    D.dl_q = ctx->dl_q.as<double>();
    D.theta = ctx->theta.as<double>();
    D.q = ctx->q.as<double>();
    D.z = ctx->r_z.as<double>();
    D.b = ctx->r_b.as<double>();
    D.ginf = ctx->r_ginf.as<double>();
    D.g2 = ctx->r_g2.as<double>();
    arb::reconstruct(s, D, rebuild);
    HIPCHK(hipGetLastError());
    std::vector<double> gi(A), gs(A);
    HIPCHK(hipMemcpyAsync(gi.data(), D.ginf, A * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(gs.data(), D.g2, A * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < A; ++a) {
        *g_inf = std::max(*g_inf, gi[a]);
        *g2 += gs[a];
    }
    return 0;
}

static int copy_state_out(arb_ctx *ctx, hipStream_t s, double *q, double *theta) {
    if (q)
        HIPCHK(hipMemcpyAsync(q, ctx->q.p, 3 * (size_t)ctx->M * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    if (theta)
        HIPCHK(hipMemcpyAsync(theta, ctx->theta.p, 4 * (size_t)ctx->M * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    return 0;
}

int arb_correct_positions(arb_ctx *ctx, double tol, int max_iter, double *q, double *theta,
                          int *iters, double *resid) {
    ARB_GUARD_BEGIN
    if (!ctx || !(tol > 0) || max_iter < 0) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(correct_run(ctx, s, tol, max_iter, iters, resid));
    TRY(refresh_geometry(ctx, s));
    TRY(copy_state_out(ctx, s, q, theta));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_reconstruct(arb_ctx *ctx, double *q, double *g_inf, double *g2) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    double gi = 0.0, gs = 0.0;
    TRY(recon_run(ctx, s, 1, &gi, &gs));
    TRY(refresh_geometry(ctx, s));
    TRY(copy_state_out(ctx, s, q, nullptr));
    HIPCHK(hipStreamSynchronize(s));
    if (g_inf) *g_inf = gi;
    if (g2) *g2 = gs;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_link_residual(arb_ctx *ctx, double *g_inf, double *g2) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    double gi = 0.0, gs = 0.0;
    TRY(recon_run(ctx, ctx->stream, 0, &gi, &gs));
    if (g_inf) *g_inf = gi;
    if (g2) *g2 = gs;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

// figures of one advance (steps 2-5 of Sec. 4.3)
struct AdvanceInfo {
    double g_inf_star = 0.0, g2_star = 0.0, corr_residual = 0.0, g_inf = 0.0;
    int corrected = 0, corr_iterations = 0;
};

// arms that change in time: checked before a step starts, so that a bad array
// leaves the context as it was
static int check_arms(arb_ctx *ctx, const arb_arms *a) {
    if (!a) return fail(ctx, ARB_E_ARG, "arms: null");
    const size_t n3 = 3 * (size_t)ctx->P;
    if (ctx->P > 0 && (!a->dl_p || !a->dl_q)) return fail(ctx, ARB_E_ARG, "arms: dl_p, dl_q required");
    if (check_finite(ctx, a->dl_p, ctx->P > 0 ? n3 : 0, "arms dl_p") ||
        check_finite(ctx, a->dl_q, ctx->P > 0 ? n3 : 0, "arms dl_q") ||
        check_finite(ctx, a->dldot_p, ctx->P > 0 ? n3 : 0, "arms dldot_p") ||
        check_finite(ctx, a->dldot_q, ctx->P > 0 ? n3 : 0, "arms dldot_q") ||
        check_finite(ctx, a->proj, ctx->P > 0 ? 3 * n3 : 0, "arms proj"))
        return ARB_E_NAN;
    return 0;
}

// the context's arms (and projections, when given; host copies and device
// arrays) become a; the constraint rows follow at the next refresh of the geometry
static int apply_arms(arb_ctx *ctx, hipStream_t s, const arb_arms *a) {
    const size_t n3 = 3 * (size_t)ctx->P;
    if (n3 == 0) return 0;
    ctx->h_dl_p.assign(a->dl_p, a->dl_p + n3);
    ctx->h_dl_q.assign(a->dl_q, a->dl_q + n3);
    if (a->dldot_p)
        ctx->h_dldot_p.assign(a->dldot_p, a->dldot_p + n3);
    else
        ctx->h_dldot_p.assign(n3, 0.0);
    if (a->dldot_q)
        ctx->h_dldot_q.assign(a->dldot_q, a->dldot_q + n3);
    else
        ctx->h_dldot_q.assign(n3, 0.0);
    TRY(upload(ctx, ctx->dl_p, ctx->h_dl_p.data(), n3, s));
    TRY(upload(ctx, ctx->dl_q, ctx->h_dl_q.data(), n3, s));
    TRY(upload(ctx, ctx->dldot_p, ctx->h_dldot_p.data(), n3, s));
    TRY(upload(ctx, ctx->dldot_q, ctx->h_dldot_q.data(), n3, s));
    if (a->proj) {
        ctx->h_proj.assign(a->proj, a->proj + 3 * n3);
        TRY(upload(ctx, ctx->proj, ctx->h_proj.data(), 3 * n3, s));
    }
    return 0;
}

// steps 2-5 of Sec. 4.3 from the context's state with body velocities Ud (device,
// 6M) over dt: every body by explicit Euler (the mean of the new tracking points
// of an articulated body is then q_COM + dt u_COM), orientations by
// theta_{w dt} . theta, rebuild, check sum g.g < delta, else correction; arms
// (may be null) are those of the end of the interval, set once the bodies moved
static int advance_dev(arb_ctx *ctx, hipStream_t s, const double *Ud, double dt, double delta,
                       double corr_tol, int corr_max_iter, AdvanceInfo *ai,
                       const arb_arms *arms = nullptr) {
    arb::euler_update(s, ctx->M, Ud, dt, ctx->q.as<double>(), ctx->theta.as<double>());
    HIPCHK(hipGetLastError());
    if (arms) TRY(apply_arms(ctx, s, arms));
    TRY(recon_run(ctx, s, 1, &ai->g_inf_star, &ai->g2_star));
    ai->g_inf = ai->g_inf_star;
    if (ctx->lasm_A > 0 && !(ai->g2_star < delta)) {
        TRY(correct_run(ctx, s, corr_tol, corr_max_iter, &ai->corr_iterations, &ai->corr_residual));
        ai->corrected = 1;
        double g2e = 0.0;
        TRY(recon_run(ctx, s, 0, &ai->g_inf, &g2e));
    }
    TRY(refresh_geometry(ctx, s));
    return 0;
}

// common checks and uploads of the time-step entry points; F, u_slip land in
// s_in / s_aux
static int step_prologue(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                         double delta, double corr_tol, int corr_max_iter) {
    if (!ctx || !F) return ARB_E_ARG;
    if (!std::isfinite(dt) || std::isnan(delta) || !(corr_tol > 0) || corr_max_iter < 0)
        return fail(ctx, ARB_E_ARG, "bad time-step arguments");
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    const int N = ctx->N, M = ctx->M;
    if (check_finite(ctx, F, 6 * (size_t)M, "F") ||
        check_finite(ctx, u_slip, u_slip ? 3 * (size_t)N : 0, "u_slip"))
        return ARB_E_NAN;
    TRY(upload(ctx, ctx->s_in, F, 6 * (size_t)M, ctx->stream));
    if (u_slip) TRY(upload(ctx, ctx->s_aux, u_slip, 3 * (size_t)N, ctx->stream));
    HIPCHK(ctx->ky.ensure(n_unknowns(ctx) * sizeof(double)));
    return 0;
}

// step 1 of Sec. 4.3 at the context's state into ky (warm: from ky's previous
// solution when its length matches)
static int step_solve(arb_ctx *ctx, hipStream_t s, bool has_slip, int warm, arb_solve_info *si) {
    const int64_t n = n_unknowns(ctx);
    const int w = (warm && ctx->ky_n == n) ? 1 : 0;
    const int rc = solve_dev(ctx, ctx->s_in.as<double>(), has_slip ? ctx->s_aux.as<double>() : nullptr,
                             ctx->ky.as<double>(), w, si, s);
    if (rc >= 0) ctx->ky_n = n;
    return rc;
}

static void fill_step_info(arb_step_info *info, int rc, const arb_solve_info &si,
                           const AdvanceInfo &ai) {
    if (!info) return;
    info->solve_status = rc;
    info->iterations = si.iterations;
    info->rel_residual = si.rel_residual;
    info->t_build_ms = si.t_build_ms;
    info->t_solve_ms = si.t_solve_ms;
    info->g_inf_star = ai.g_inf_star;
    info->g2_star = ai.g2_star;
    info->corrected = ai.corrected;
    info->corr_iterations = ai.corr_iterations;
    info->corr_residual = ai.corr_residual;
    info->g_inf = ai.g_inf;
}

static int step_euler(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                      double delta, double corr_tol, int corr_max_iter, int warm,
                      const arb_arms *end, double *q, double *theta, double *U,
                      arb_step_info *info) {
    TRY(step_prologue(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter));
    hipStream_t s = ctx->stream;
    arb_solve_info si{};
    const int rc = step_solve(ctx, s, u_slip != nullptr, warm, &si);
    if (rc < 0) return rc;
    const double *Ud = ctx->ky.as<double>() + u_offset(ctx);
    AdvanceInfo ai;
    TRY(advance_dev(ctx, s, Ud, dt, delta, corr_tol, corr_max_iter, &ai, end));
    TRY(copy_state_out(ctx, s, q, theta));
    if (U)
        HIPCHK(hipMemcpyAsync(U, Ud, 6 * (size_t)ctx->M * sizeof(double), hipMemcpyDeviceToHost,
                              s));
    HIPCHK(hipStreamSynchronize(s));
    fill_step_info(info, rc, si, ai);
    return rc;
}

static int step_midpoint(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                         double delta, double corr_tol, int corr_max_iter, int warm,
                         const arb_arms *mid, const arb_arms *end, double *q, double *theta,
                         double *U, arb_step_info *info) {
    TRY(step_prologue(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter));
    hipStream_t s = ctx->stream;
    const int M = ctx->M;
    // the initial state, to which the full step returns
    HIPCHK(ctx->q0.ensure(3 * (size_t)M * sizeof(double)));
    HIPCHK(ctx->th0.ensure(4 * (size_t)M * sizeof(double)));
    HIPCHK(hipMemcpyAsync(ctx->q0.p, ctx->q.p, 3 * (size_t)M * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->th0.p, ctx->theta.p, 4 * (size_t)M * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    const double *Ud = ctx->ky.as<double>() + u_offset(ctx);
    // U^k, half step to the midpoint state
    arb_solve_info s0{};
    const int rc0 = step_solve(ctx, s, u_slip != nullptr, warm, &s0);
    if (rc0 < 0) return rc0;
    AdvanceInfo ah;
    TRY(advance_dev(ctx, s, Ud, 0.5 * dt, delta, corr_tol, corr_max_iter, &ah, mid));
    // U^(k+1/2) at the midpoint state, warm-started from U^k's solution
    arb_solve_info s1{};
    const int rc1 = step_solve(ctx, s, u_slip != nullptr, 1, &s1);
    if (rc1 < 0) return rc1;
    // full step from the initial state
    HIPCHK(hipMemcpyAsync(ctx->q.p, ctx->q0.p, 3 * (size_t)M * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->theta.p, ctx->th0.p, 4 * (size_t)M * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    AdvanceInfo af;
    TRY(advance_dev(ctx, s, Ud, dt, delta, corr_tol, corr_max_iter, &af, end));
    TRY(copy_state_out(ctx, s, q, theta));
    if (U) HIPCHK(hipMemcpyAsync(U, Ud, 6 * (size_t)M * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    arb_solve_info st = s1;
    st.iterations = s0.iterations + s1.iterations;
    st.rel_residual = std::max(s0.rel_residual, s1.rel_residual);
    st.t_build_ms = s0.t_build_ms + s1.t_build_ms;
    st.t_solve_ms = s0.t_solve_ms + s1.t_solve_ms;
    af.corrected |= ah.corrected;
    af.corr_iterations = std::max(af.corr_iterations, ah.corr_iterations);
    // a solve that did not converge outranks other warnings
    const int rc = (rc0 == ARB_W_NOT_CONVERGED || rc1 == ARB_W_NOT_CONVERGED)
                       ? ARB_W_NOT_CONVERGED
                       : (rc0 > 0 ? rc0 : rc1);
    fill_step_info(info, rc, st, af);
    return rc;
}

int arb_step_euler(arb_ctx *ctx, const double *F, const double *u_slip, double dt, double delta,
                   double corr_tol, int corr_max_iter, int warm, double *q, double *theta,
                   double *U, arb_step_info *info) {
    ARB_GUARD_BEGIN
    return step_euler(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter, warm, nullptr, q,
                      theta, U, info);
    ARB_GUARD_END(ctx)
}

int arb_step_euler_arms(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                        double delta, double corr_tol, int corr_max_iter, int warm,
                        const arb_arms *end, double *q, double *theta, double *U,
                        arb_step_info *info) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    TRY(check_arms(ctx, end));
    return step_euler(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter, warm, end, q, theta,
                      U, info);
    ARB_GUARD_END(ctx)
}

int arb_step_midpoint(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                      double delta, double corr_tol, int corr_max_iter, int warm, double *q,
                      double *theta, double *U, arb_step_info *info) {
    ARB_GUARD_BEGIN
    return step_midpoint(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter, warm, nullptr,
                         nullptr, q, theta, U, info);
    ARB_GUARD_END(ctx)
}

int arb_step_midpoint_arms(arb_ctx *ctx, const double *F, const double *u_slip, double dt,
                           double delta, double corr_tol, int corr_max_iter, int warm,
                           const arb_arms *mid, const arb_arms *end, double *q, double *theta,
                           double *U, arb_step_info *info) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    TRY(check_arms(ctx, mid));
    TRY(check_arms(ctx, end));
    return step_midpoint(ctx, F, u_slip, dt, delta, corr_tol, corr_max_iter, warm, mid, end, q,
                         theta, U, info);
    ARB_GUARD_END(ctx)
}

// parameter block: allocated once with identity standardisation
static int mlp_alloc(arb_ctx *ctx) {
    if (ctx->mlp_params.p) return 0;
    HIPCHK(ctx->mlp_params.ensure((size_t)arb::mlp_param_bytes()));
    HIPCHK(hipMemsetAsync(ctx->mlp_params.p, 0, (size_t)arb::mlp_param_bytes(), ctx->stream));
    const float z[32] = {0}, o[32] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                      1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    arb::mlp_set_scaling(ctx->stream, ctx->mlp_params.p, z, o, z, o);
    return 0;
}

int arb_mlp_set_scaling(arb_ctx *ctx, const float *in_mu, const float *in_sd, const float *out_mu,
                        const float *out_sd) {
    ARB_GUARD_BEGIN
    if (!ctx || !in_mu || !in_sd || !out_mu || !out_sd) return ARB_E_ARG;
    for (int k = 0; k < 7; ++k)
        if (!(in_sd[k] > 0) || !std::isfinite(in_mu[k])) return fail(ctx, ARB_E_ARG, "bad input scaling");
    for (int k = 0; k < 21; ++k)
        if (!(out_sd[k] > 0) || !std::isfinite(out_mu[k])) return fail(ctx, ARB_E_ARG, "bad output scaling");
    HIPCHK(hipSetDevice(ctx->opt.device));
    TRY(mlp_alloc(ctx));
    arb::mlp_set_scaling(ctx->stream, ctx->mlp_params.p, in_mu, in_sd, out_mu, out_sd);
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mlp_set_params(arb_ctx *ctx, int n, const float *params) {
    ARB_GUARD_BEGIN
    if (!ctx || !params) return ARB_E_ARG;
    if (n != arb::mlp_n_params()) return fail(ctx, ARB_E_ARG, "wrong parameter count");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(params[k])) return fail(ctx, ARB_E_NAN, "parameters not finite");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(mlp_alloc(ctx));
    HIPCHK(hipMemsetAsync(ctx->mlp_params.p, 0, (size_t)arb::mlp_state_bytes(), s));
    HIPCHK(hipMemcpyAsync(ctx->mlp_params.p, params, (size_t)n * sizeof(float),
                          hipMemcpyHostToDevice, s));
    arb::mlp_refresh(s, ctx->mlp_params.p);
    HIPCHK(hipStreamSynchronize(s));
    ctx->mlp_ready = true;
    ctx->mlp_step = 0;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mlp_get_params(arb_ctx *ctx, int n, float *params) {
    ARB_GUARD_BEGIN
    if (!ctx || !params) return ARB_E_ARG;
    if (!ctx->mlp_ready) return fail(ctx, ARB_E_ARG, "parameters not set");
    if (n != arb::mlp_n_params()) return fail(ctx, ARB_E_ARG, "wrong parameter count");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipMemcpyAsync(params, ctx->mlp_params.p, (size_t)n * sizeof(float),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mlp_forward(arb_ctx *ctx, int B, const float *X, float *Y) {
    ARB_GUARD_BEGIN
    if (!ctx || B <= 0 || !X || !Y) return ARB_E_ARG;
    if (!ctx->mlp_ready) return fail(ctx, ARB_E_ARG, "parameters not set");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    const int Bp = (B + 15) / 16 * 16;
    TRY(mlp_ensure_ws(ctx, Bp));
    TRY(upload(ctx, ctx->mlp_x, X, (size_t)B * 7, s));
    float *Yd = arb::mlp_forward(s, ctx->mlp_params.p, ctx->mlp_ws.p, B, Bp, ctx->mlp_x.as<float>());
    arb::mlp_destandardize(s, ctx->mlp_params.p, B, Yd);
    std::vector<float> tmp((size_t)Bp * 32);
    HIPCHK(hipMemcpyAsync(tmp.data(), Yd, tmp.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < 21; ++k) Y[(size_t)b * 21 + k] = tmp[(size_t)b * 32 + k];
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

static int mlp_grad_dev(arb_ctx *ctx, hipStream_t s, int B, const float *Xd, const float *Td,
                        double *loss) {
    const int Bp = (B + 15) / 16 * 16;
    TRY(mlp_ensure_ws(ctx, Bp));
    double *lp = nullptr;
    const int nlp = arb::mlp_backward(s, ctx->mlp_params.p, ctx->mlp_ws.p, B, Bp, Xd, Td, &lp);
    if (loss) {
        std::vector<double> h(nlp);
        HIPCHK(hipMemcpyAsync(h.data(), lp, nlp * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double t = 0.0;
        for (double v : h) t += v;
        *loss = t / ((double)B * 21.0);
    }
    return 0;
}

int arb_mlp_grad(arb_ctx *ctx, int B, const float *X, const float *T, float *grad, double *loss) {
    ARB_GUARD_BEGIN
    if (!ctx || B <= 0 || !X || !T || !grad) return ARB_E_ARG;
    if (!ctx->mlp_ready) return fail(ctx, ARB_E_ARG, "parameters not set");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    TRY(upload(ctx, ctx->mlp_x, X, (size_t)B * 7, s));
    TRY(upload(ctx, ctx->mlp_t, T, (size_t)B * 21, s));
    TRY(mlp_grad_dev(ctx, s, B, ctx->mlp_x.as<float>(), ctx->mlp_t.as<float>(), loss));
    const int n = arb::mlp_n_params();
    const float *G = ctx->mlp_params.as<float>() + 3 * (size_t)n;
    HIPCHK(hipMemcpyAsync(grad, G, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mlp_train_step_dev(arb_ctx *ctx, int B, const float *X_dev, const float *T_dev, float lr,
                           double *loss, void *stream) {
    ARB_GUARD_BEGIN
    if (!ctx || B <= 0 || !X_dev || !T_dev || !(lr > 0)) return ARB_E_ARG;
    if (!ctx->mlp_ready) return fail(ctx, ARB_E_ARG, "parameters not set");
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = pick(ctx, stream);
    TRY(mlp_grad_dev(ctx, s, B, X_dev, T_dev, loss));
    arb::mlp_adam(s, ctx->mlp_params.p, lr, ++ctx->mlp_step);
    HIPCHK(hipGetLastError());
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_mlp_features(arb_ctx *ctx, float *X) {
    ARB_GUARD_BEGIN
    if (!ctx || !X) return ARB_E_ARG;
    TRY(ready(ctx));
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx->mlp_x.ensure((size_t)ctx->M * 7 * sizeof(float)));
    arb::mlp_features(s, ctx->M, ctx->q.as<double>(), ctx->theta.as<double>(),
                      ctx->body_type_d.as<int>(), ctx->opt.a, ctx->mlp_x.as<float>());
    HIPCHK(hipMemcpyAsync(X, ctx->mlp_x.p, (size_t)ctx->M * 7 * sizeof(float),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_body_mobility(arb_ctx *ctx, double *Nt, float *target) {
    ARB_GUARD_BEGIN
    if (!ctx || (!Nt && !target)) return ARB_E_ARG;
    HIPCHK(hipSetDevice(ctx->opt.device));
    hipStream_t s = ctx->stream;
    const int rc = precond_build_exact(ctx, s);
    if (rc < 0) return rc;
    const int M = ctx->M;
    if (Nt)
        HIPCHK(hipMemcpyAsync(Nt, ctx->Nt.p, 36 * (size_t)M * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    if (target) {
        HIPCHK(ctx->mlp_t.ensure((size_t)M * 21 * sizeof(float)));
        HIPCHK(hipMemsetAsync(ctx->status.as<int>() + 5, 0, sizeof(int), s));
        arb::mlp_targets(s, M, ctx->Nt.as<double>(), ctx->opt.a, ctx->opt.eta, ctx->mlp_t.as<float>(),
                         ctx->status.as<int>() + 5);
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ctx->status.as<int>() + 5, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(target, ctx->mlp_t.p, (size_t)M * 21 * sizeof(float),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad) return fail(ctx, ARB_E_NOT_SPD, "a body mobility is not positive definite");
    }
    HIPCHK(hipStreamSynchronize(s));
    return rc;
    ARB_GUARD_END(ctx)
}

int arb_profile(arb_ctx *ctx, int enable) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    ctx->prof = enable != 0;
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

int arb_profile_read(arb_ctx *ctx, double *pair_ms, int *pair_launches) {
    ARB_GUARD_BEGIN
    if (!ctx) return ARB_E_ARG;
    HIPCHK(hipSetDevice(ctx->opt.device));
    double tot = 0.0;
    for (auto &e : ctx->prof_ev) {
        HIPCHK(hipEventSynchronize(e.second));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
        tot += ms;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (pair_ms) *pair_ms = tot;
    if (pair_launches) *pair_launches = (int)ctx->prof_ev.size();
    ctx->prof_ev.clear();
    return ARB_OK;
    ARB_GUARD_END(ctx)
}

}  // extern "C"
