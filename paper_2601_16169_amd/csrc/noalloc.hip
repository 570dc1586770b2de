// sqd_sigma_noalloc: the product of sqd_sigma for callers that cannot call the
// device allocator (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  Its scratch -- the transposed input of the
// alpha-alpha term and that term's output, plus the FP32 copies of the FP32
// path -- lives in one statically sized device array, `scratch`, instead of
// the context's grown-on-demand buffer, and the alpha-beta term runs the
// row-staged kernel, which keeps no intermediate.
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress (at context creation,
// with the device current) and only that address is handed to kernels.
#include <mutex>

#include "sqd_internal.h"

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

// Shared by every call on a device; holds the last call's data.
static __device__ __align__(256) unsigned char scratch[SQD_NOALLOC_SCRATCH_BYTES];

// Look up this device's copy of `scratch` (the device must be current).
int sqd_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SQD_E_LIMIT;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch_dev[device]) return SQD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return SQD_E_HIP;
    }
    g_scratch_dev[device] = p;
    return SQD_OK;
}

extern "C" int sqd_sigma_noalloc(sqd_ctx* ctx, const sqd_space* spc, const double* c, double* sigma,
                                 int precision, unsigned mask) {
    if (!ctx || !spc || !c || !sigma) return SQD_E_INVALID_ARG;
    sqd_space* sp = const_cast<sqd_space*>(spc);
    if (sp->ctx != ctx) return sqd_fail(ctx, SQD_E_INVALID_ARG, "space belongs to another context");
    if (ctx->norb != sp->norb) return sqd_fail(ctx, SQD_E_STATE, "integrals changed norb since the space was built");
    if (precision != SQD_FP64 && precision != SQD_FP32) return sqd_fail(ctx, SQD_E_INVALID_ARG, "bad precision");
    if (mask == 0 || (mask & ~SQD_TERM_ALL)) return sqd_fail(ctx, SQD_E_INVALID_ARG, "bad terms mask");
    if (c == sigma) return sqd_fail(ctx, SQD_E_INVALID_ARG, "c and sigma must be distinct buffers");
    if (sp->dim > SQD_NOALLOC_MAX_DIM)
        return sqd_fail(ctx, SQD_E_LIMIT, "dimension " + std::to_string(sp->dim) + " above the no-allocation limit " +
                                              std::to_string((long long)SQD_NOALLOC_MAX_DIM));
    void* buf = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) buf = g_scratch_dev[ctx->device];
    }
    if (!buf) return sqd_fail(ctx, SQD_E_STATE, "static product scratch has no device address on this device");
    SQD_HIP(ctx, hipSetDevice(ctx->device));
    // windowed tables for long same-spin rows are built (allocated) by the
    // space's first allocating product with that term
    if (!sqd_space_built_for(ctx, sp, precision, mask))
        return sqd_fail(ctx, SQD_E_STATE, "windowed same-spin tables not built: call sqd_sigma on this space first");
    // values and diagonal are refreshed in place after a Hamiltonian change
    // (kernels and a synchronisation, no allocation); under capture they must
    // already be current
    if ((sp->values_version != ctx->ham_version || sp->diag_version != ctx->ham_version) && sqd_capturing(ctx))
        return sqd_fail(ctx, SQD_E_STATE, "integrals changed since the last product on this space");
    // the timers create events on demand: off for this call
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    const int rc = sqd_sigma_impl(ctx, sp, c, sigma, precision, mask, SQD_AB_DIRECT, nullptr, nullptr, buf,
                                  (size_t)SQD_NOALLOC_SCRATCH_BYTES);
    ctx->profiling = prof;
    return rc;
}
