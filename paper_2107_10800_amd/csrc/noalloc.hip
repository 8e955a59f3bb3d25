// Allocation-free blob mobility product (arb_rpy_apply_noalloc_dev in arb.h).
//
// The same product as arb_rpy_apply_dev (u = M lambda over loose blobs, Sec. 2.3
// Eq. RPY, unbounded or above the wall) on the target-parallel kernels of
// pair.hip, with every intermediate buffer in one file-scope device array:
//
//   [ p64: N double4 | hi: N float4 | lo: N float4 ]  staged positions, 64 B/blob
//   [ partial: slices x 3 x N doubles ]               per-slice sums
//
// The positions region is sized for ARB_NOALLOC_MAX_BLOBS blobs, the partial
// region for four source slices at that size (more slices at smaller sizes).
// Every slice stores (does not accumulate) its sums, so nothing has to start
// at zero.  One copy of the array exists per device; calls that overlap on one
// device race on it.
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kPosBytes =
    (size_t)ARB_NOALLOC_MAX_BLOBS * (sizeof(double4) + 2 * sizeof(float4));
constexpr size_t kPartialDoubles = (size_t)4 * 3 * ARB_NOALLOC_MAX_BLOBS;
constexpr size_t kScratchBytes = kPosBytes + kPartialDoubles * sizeof(double);
static_assert(kPosBytes % 256 == 0, "partial region must stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};  // device address of scratch, per device
int g_state[kMaxDevices] = {};  // 0 not looked up, 1 found, -1 lookup failed

int fail(arb_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

}  // namespace

namespace arb {

// Looks up this device's copy of the scratch array; call with `device` current.
// Host code never uses the array's name as an address: only the pointer found
// here.  Returns 0 when the address is known.
int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_state[device] != 0) return g_state[device] == 1 ? 0 : -1;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        g_state[device] = -1;
        return -1;
    }
    g_ptr[device] = p;
    g_state[device] = 1;
    return 0;
}

}  // namespace arb

static int rpy_apply_noalloc(arb_ctx *ctx, int N, const double *pos_dev,
                             const double *lambda_dev, double *u_dev, void *stream) {
    if (!ctx) return ARB_E_ARG;
    if (N < 0 || (N > 0 && (!pos_dev || !lambda_dev || !u_dev)))
        return fail(ctx, ARB_E_ARG, "arb_rpy_apply_noalloc_dev: bad size or null pointer");
    if (N > ARB_NOALLOC_MAX_BLOBS)
        return fail(ctx, ARB_E_ARG,
                    "arb_rpy_apply_noalloc_dev: " + std::to_string(N) +
                        " blobs exceed the allocation-free maximum of " +
                        std::to_string(ARB_NOALLOC_MAX_BLOBS));
    if (ctx->opt.pair_kernel == ARB_PAIR_FMM)
        return fail(ctx, ARB_E_ARG,
                    "arb_rpy_apply_noalloc_dev: the fast product needs allocated tree buffers");
    if (N == 0) return ARB_OK;
    const int dev = ctx->opt.device;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess)
        return fail(ctx, ARB_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    if (arb::noalloc_setup(dev) != 0)
        return fail(ctx, ARB_E_DEVICE,
                    "arb_rpy_apply_noalloc_dev: hipGetSymbolAddress of the scratch array failed");
    unsigned char *base = static_cast<unsigned char *>(g_ptr[dev]);
    double4 *p64 = reinterpret_cast<double4 *>(base);
    float4 *hi = reinterpret_cast<float4 *>(p64 + N);
    float4 *lo = hi + N;
    double *partial = reinterpret_cast<double *>(base + kPosBytes);
    // slices as the options give them, else the heuristic; at most what the
    // partial region holds at this size
    int slices = ctx->opt.slices > 0 ? ctx->opt.slices : arb::heuristic_slices(N);
    const int cap = (int)(kPartialDoubles / (3 * (size_t)N));
    slices = std::max(1, std::min(slices, cap));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    arb::prep_positions(s, N, pos_dev, ctx->opt.a, p64, hi, lo, nullptr, nullptr);
    const int used = arb::pair_partial(s, ctx->opt.precision, ctx->opt.wall != 0, N, p64, hi,
                                       lo, lambda_dev, nullptr, ctx->opt.a, slices, partial);
    // FP32 sums are in units of the blob radius: M(a) = M_{a=1}(r / a) / a
    const double scale = 1.0 / (8.0 * arb::kPi * ctx->opt.eta) /
                         (ctx->opt.precision == ARB_FP32C ? ctx->opt.a : 1.0);
    arb::pair_reduce(s, N, used, partial, scale, u_dev, nullptr, nullptr, nullptr, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess)
        return fail(ctx, ARB_E_DEVICE, std::string("pair launch: ") + hipGetErrorString(e));
    return ARB_OK;
}

extern "C" int arb_rpy_apply_noalloc_dev(arb_ctx *ctx, int N, const double *pos_dev,
                                         const double *lambda_dev, double *u_dev,
                                         void *stream) {
    try {
        return rpy_apply_noalloc(ctx, N, pos_dev, lambda_dev, u_dev, stream);
    } catch (...) {  // an error message that could not be formed
        return ARB_E_HOST;
    }
}
