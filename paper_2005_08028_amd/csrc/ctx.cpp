// Context lifetime, error reporting and scratch management of libscitv.
#include <hip/hip_runtime_api.h>

#include <new>
#include <string>

#include "sci_internal.h"

namespace sci {

int fail_hip(sci_ctx *ctx, hipError_t e, const char *what)
{
    if (ctx) ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SCI_ERR_NOMEM : SCI_ERR_HIP;
}

int fail(sci_ctx *ctx, int status, const std::string &msg)
{
    if (ctx) ctx->last_error = msg;
    return status;
}

int check_launch(sci_ctx *ctx, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(ctx, e, what);
    return SCI_OK;
}

// Grow a scratch slot to at least `bytes` (rounded up to 256). Growing
// waits for `stream` so that queued work never sees its buffer freed.
int ensure_ws(sci_ctx *ctx, BufSlot slot, size_t bytes, hipStream_t stream)
{
    Buf &b = ctx->ws[slot];
    bytes = (bytes + 255) & ~(size_t)255;
    if (b.bytes >= bytes) return SCI_OK;
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return fail_hip(ctx, e, "hipDeviceSynchronize");
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
        // graphs captured earlier may point at the freed buffer
        for (auto &kv : ctx->graphs) destroy_graph(kv.second);
        ctx->graphs.clear();
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return fail_hip(ctx, e, "hipMalloc(scratch)");
    }
    b.bytes = bytes;
    return SCI_OK;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t dual_elem_bytes(int dual_dtype) { return dual_dtype == SCI_DUAL_F32 ? 4 : 2; }

int drop_graphs(sci_ctx *ctx)
{
    if (ctx->graphs.empty()) return SCI_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail_hip(ctx, e, "hipDeviceSynchronize");
    for (auto &kv : ctx->graphs) destroy_graph(kv.second);
    ctx->graphs.clear();
    return SCI_OK;
}

void destroy_graph(GraphEntry &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.owned) (void)hipFree(g.owned);
    g.exec = nullptr;
    g.owned = nullptr;
}

static hipEvent_t pool_event(sci_ctx *ctx)
{
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDefault) != hipSuccess) return nullptr;
        ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
}

ProfScope::ProfScope(sci_ctx *ctx, int family, hipStream_t s) : ctx_(ctx), family_(family), s_(s)
{
    if (!ctx_->prof_on || ctx_->capturing) return;
    a_ = pool_event(ctx_);
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    hipEvent_t b = pool_event(ctx_);
    if (b && hipEventRecord(b, s_) == hipSuccess) ctx_->prof.push_back(ProfRec{family_, a_, b});
}

} // namespace sci

extern "C" {

int sci_create(sci_ctx **out, int device)
{
    if (!out) return SCI_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SCI_ERR_INVALID_ARG;
    sci_ctx *ctx = new (std::nothrow) sci_ctx();
    if (!ctx) return SCI_ERR_NOMEM;
    ctx->device = device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete ctx;
        return SCI_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    if (sci::noalloc_scratch_lookup(device, &ctx->noalloc_scratch) != SCI_OK) {
        delete ctx;
        return SCI_ERR_HIP;
    }
    e = hipHostMalloc((void **)&ctx->host_scalars, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return SCI_ERR_NOMEM;
    }
    e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipHostFree(ctx->host_scalars);
        delete ctx;
        return SCI_ERR_HIP;
    }
    *out = ctx;
    return SCI_OK;
}

void sci_destroy(sci_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->graphs) sci::destroy_graph(kv.second);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto &b : ctx->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->host_scalars) (void)hipHostFree(ctx->host_scalars);
    delete ctx;
}

const char *sci_status_string(int status)
{
    switch (status) {
    case SCI_OK: return "ok";
    case SCI_NOT_CONVERGED: return "duality-gap tolerance not met at the iteration cap (outputs written)";
    case SCI_ERR_INVALID_ARG: return "invalid argument";
    case SCI_ERR_ALIAS: return "an output overlaps an input";
    case SCI_ERR_NOMEM: return "out of device memory";
    case SCI_ERR_HIP: return "HIP runtime error";
    case SCI_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *sci_last_error(const sci_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int sci_profile_enable(sci_ctx *ctx, int enable)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    if (enable) {
        hipError_t e = hipDeviceSynchronize(); // recorded events may still be pending
        if (e != hipSuccess) return sci::fail_hip(ctx, e, "hipDeviceSynchronize");
        ctx->prof.clear();
        ctx->ev_used = 0;
    }
    ctx->prof_on = enable != 0;
    return SCI_OK;
}

int sci_profile_read(sci_ctx *ctx, const char *family, int64_t *launches, double *total_ms)
{
    static const char *names[sci::PF_COUNT] = {"fgp_stream", "fgp_fused", "tv_theta", "project", "setup"};
    if (!ctx || !family) return SCI_ERR_INVALID_ARG;
    int fam = -1;
    for (int k = 0; k < sci::PF_COUNT; ++k)
        if (std::string(family) == names[k]) fam = k;
    if (fam < 0) return sci::fail(ctx, SCI_ERR_INVALID_ARG, std::string("unknown kernel family ") + family);
    int64_t n = 0;
    double ms = 0.0;
    for (const sci::ProfRec &r : ctx->prof) {
        if (r.family != fam) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return sci::fail_hip(ctx, e, "hipEventSynchronize");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) return sci::fail_hip(ctx, e, "hipEventElapsedTime");
        ms += t;
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return SCI_OK;
}

} // extern "C"
