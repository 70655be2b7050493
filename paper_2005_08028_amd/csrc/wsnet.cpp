// Host side of the warm-start network: parameters, activation scratch,
// forward, gradients (all layers; dual-space MSE or theta-space loss), Adam
// steps, and the projected dual field handed to the FGP denoiser as its
// starting point.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <new>
#include <string>

#include "sci_internal.h"
#include "sci_wsnet.h"

using namespace sci;

struct sci_wsnet {
    int c_in = 1;  // 1: x only; 3: x and a base dual (the prediction is added to it)
    int c_out = 2;
    int loss = SCI_WSNET_LOSS_DUAL;
    int device = 0;
    int64_t step = 0;
    // per layer: fp32 master params / Adam moments / gradient in [28][16][16]
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    // per layer: bf16 packs Wk[27][16][16], WkT (mirrored, transposed), fp32 bias[16]
    uint16_t *Wk = nullptr, *WkT = nullptr;
    float *bias = nullptr;
    // activations for the largest volume seen
    size_t vcap = 0;
    uint16_t *act[kNetLayers] = {nullptr, nullptr, nullptr, nullptr}; // layer inputs a1..a3 (a0: the fp32 planes)
    uint8_t *sgn[kNetLayers] = {nullptr, nullptr, nullptr, nullptr};  // sign bytes [V][4] of a1..a3 (training)
    uint16_t *dA = nullptr, *dB = nullptr;                            // gradient ping-pong
    float *y = nullptr;                                               // last layer output [c_out][V]
    float *gth = nullptr;                                             // theta-loss D^T r [V]
    float *wpart = nullptr;                                           // wgrad partials, per layer
    double *lpart = nullptr;                                          // loss partials (+ result)
};

namespace {

int net_fail(sci_ctx *ctx, hipError_t e, const char *what) { return fail_hip(ctx, e, what); }

void free_acts(sci_wsnet *n)
{
    for (auto &a : n->act) {
        if (a) (void)hipFree(a);
        a = nullptr;
    }
    for (auto &a : n->sgn) {
        if (a) (void)hipFree(a);
        a = nullptr;
    }
    if (n->dA) (void)hipFree(n->dA);
    if (n->dB) (void)hipFree(n->dB);
    if (n->y) (void)hipFree(n->y);
    if (n->gth) (void)hipFree(n->gth);
    n->dA = n->dB = nullptr;
    n->y = nullptr;
    n->gth = nullptr;
    n->vcap = 0;
}

int ensure_acts(sci_ctx *ctx, sci_wsnet *n, size_t V, hipStream_t s)
{
    if (n->vcap >= V) return SCI_OK;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return net_fail(ctx, e, "hipStreamSynchronize");
    free_acts(n);
    const size_t ab = V * 16 * sizeof(uint16_t);
    for (int l = 1; l < kNetLayers; ++l)
        if ((e = hipMalloc(&n->act[l], ab)) != hipSuccess || (e = hipMalloc(&n->sgn[l], V * 4)) != hipSuccess)
            return net_fail(ctx, e, "hipMalloc(activations)");
    if ((e = hipMalloc(&n->dA, ab)) != hipSuccess || (e = hipMalloc(&n->dB, ab)) != hipSuccess ||
        (e = hipMalloc(&n->y, V * (size_t)n->c_out * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&n->gth, V * sizeof(float))) != hipSuccess)
        return net_fail(ctx, e, "hipMalloc(activations)");
    n->vcap = V;
    return SCI_OK;
}

int check_net_args(sci_ctx *ctx, sci_wsnet *n, const sci_dims &d, const float *X)
{
    if (!ctx || !n) return SCI_ERR_INVALID_ARG;
    if (d.nx < 1 || d.ny < 1 || d.B < 1 || (int64_t)d.nx * d.ny * d.B >= ((int64_t)1 << 31))
        return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: bad dims");
    if (!X) return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: null input");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipSetDevice");
    }
    return SCI_OK;
}

// a1 = relu(conv_0(X [, base])), read from the fp32 planes; a_{l+1} =
// relu(conv_l(a_l)); the last layer writes the raw output planes y or, when
// `dual` is given (a pointwise projection: ATV, ITV2D), the projected
// (base +) output straight into it. The sign bytes of a1..a3 (the ReLU masks
// of the data gradients) are written only for the gradients.
void forward(sci_wsnet *n, const sci_dims &d, const float *X, const float *P_base, bool for_grads, float *dual,
             int tv, hipStream_t s)
{
    const float *base = n->c_in == 3 ? P_base : nullptr;
    wsnet_conv_input(d.nx, d.ny, d.B, X, base, n->Wk, n->bias, n->act[1], for_grads ? n->sgn[1] : nullptr, s);
    for (int l = 1; l < kNetLayers - 1; ++l)
        wsnet_conv(d.nx, d.ny, d.B, n->act[l], n->Wk + (size_t)l * 27 * 256, n->bias + l * 16, true, nullptr,
                   n->act[l + 1], for_grads ? n->sgn[l + 1] : nullptr, s);
    const int l = kNetLayers - 1;
    const uint16_t *Wk = n->Wk + (size_t)l * 27 * 256;
    if (dual) wsnet_conv_dual(d.nx, d.ny, d.B, n->act[l], Wk, n->bias + l * 16, tv, base, dual, s);
    else wsnet_conv_out(d.nx, d.ny, d.B, n->act[l], Wk, n->bias + l * 16, n->c_out, n->y, s);
}

// loss and gradients of every layer into n->g
void backward(sci_ctx *ctx, sci_wsnet *n, const sci_dims &d, const float *X, const float *base, const float *target,
              hipStream_t s)
{
    const int nb = wsnet_reduce_blocks();
    const float *b = n->c_in == 3 ? base : nullptr;
    if (n->loss == SCI_WSNET_LOSS_THETA)
        wsnet_loss_theta(d.nx, d.ny, d.B, n->y, b, target, n->gth, n->dA, n->lpart, n->lpart + nb, s);
    else
        wsnet_loss(d.nx, d.ny, d.B, n->c_out, n->y, b, target, n->dA, n->lpart, n->lpart + nb, s);
    uint16_t *dcur = n->dA, *dnext = n->dB;
    int groups = 0;
    for (int l = kNetLayers - 1; l >= 0; --l) {
        // the first layer's input straight from the fp32 planes, as its forward reads it
        float *part = n->wpart + (size_t)l * wsnet_wgrad_groups() * kNetSlots;
        groups = l == 0 ? wsnet_wgrad(d.nx, d.ny, d.B, dcur, nullptr, X, b, part, s)
                        : wsnet_wgrad(d.nx, d.ny, d.B, dcur, n->act[l], nullptr, nullptr, part, s);
        if (l > 0) {
            // d a_l = conv^T(d y_l), masked by the ReLU of a_l (its sign bytes)
            wsnet_conv(d.nx, d.ny, d.B, dcur, n->WkT + (size_t)l * 27 * 256, nullptr, false, n->sgn[l], dnext,
                       nullptr, s);
            std::swap(dcur, dnext);
        }
    }
    wsnet_wgrad_reduce(kNetLayers, groups, n->wpart, n->g, s);
    (void)ctx;
}

// the summed loss divided by its normaliser: c_out V entries (dual MSE) or
// V voxels (theta)
double loss_value(const sci_wsnet *n, double sum, size_t V)
{
    return n->loss == SCI_WSNET_LOSS_THETA ? sum / (double)V : sum / ((double)n->c_out * (double)V);
}

void adam(sci_wsnet *n, float lr, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int64_t t = n->step;
    const float c1 = lr != 0.0f ? (float)(1.0 - std::pow(0.9, (double)t)) : 1.0f;
    const float c2 = lr != 0.0f ? (float)(1.0 - std::pow(0.999, (double)t)) : 1.0f;
    wsnet_adam(kNetLayers, n->c_in, n->c_out, lr, b1, b2, eps, c1, c2, n->g, n->w, n->m, n->v, n->Wk, n->WkT, n->bias,
               s);
}

} // namespace

int sci::wsnet_input_channels(const sci_wsnet *n) { return n ? n->c_in : 0; }

extern "C" {

int sci_wsnet_create(sci_ctx *ctx, int32_t c_in, int32_t c_out, sci_wsnet **out)
{
    if (!ctx || !out) return SCI_ERR_INVALID_ARG;
    *out = nullptr;
    if (c_in != 1 && c_in != 3) return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: c_in is 1 or 3");
    if (c_out < 1 || c_out > kNetHidden || (c_in == 3 && c_out != 2))
        return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: c_out in 1..16 (2 with a base dual)");
    sci_wsnet *n = new (std::nothrow) sci_wsnet();
    if (!n) return SCI_ERR_NOMEM;
    n->c_in = c_in;
    n->c_out = c_out;
    n->device = ctx->device;
    const size_t pb = (size_t)kNetLayers * kNetSlots * sizeof(float);
    hipError_t e;
    if ((e = hipMalloc(&n->w, pb)) != hipSuccess || (e = hipMalloc(&n->m, pb)) != hipSuccess ||
        (e = hipMalloc(&n->v, pb)) != hipSuccess || (e = hipMalloc(&n->g, pb)) != hipSuccess ||
        (e = hipMalloc(&n->Wk, (size_t)kNetLayers * 27 * 256 * 2)) != hipSuccess ||
        (e = hipMalloc(&n->WkT, (size_t)kNetLayers * 27 * 256 * 2)) != hipSuccess ||
        (e = hipMalloc(&n->bias, (size_t)kNetLayers * 16 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&n->wpart, (size_t)kNetLayers * wsnet_wgrad_groups() * kNetSlots * sizeof(float))) !=
            hipSuccess ||
        (e = hipMalloc(&n->lpart, ((size_t)wsnet_reduce_blocks() + 8) * sizeof(double))) != hipSuccess) {
        sci_wsnet_destroy(n);
        return fail_hip(ctx, e, "hipMalloc(wsnet)");
    }
    if ((e = hipMemset(n->w, 0, pb)) != hipSuccess || (e = hipMemset(n->m, 0, pb)) != hipSuccess ||
        (e = hipMemset(n->v, 0, pb)) != hipSuccess || (e = hipMemset(n->g, 0, pb)) != hipSuccess) {
        sci_wsnet_destroy(n);
        return fail_hip(ctx, e, "hipMemset(wsnet)");
    }
    adam(n, 0.0f, nullptr); // pack the (zero) weights
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        sci_wsnet_destroy(n);
        return fail_hip(ctx, e, "wsnet init");
    }
    *out = n;
    return SCI_OK;
}

void sci_wsnet_destroy(sci_wsnet *n)
{
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipDeviceSynchronize();
    free_acts(n);
    for (void *p : {(void *)n->w, (void *)n->m, (void *)n->v, (void *)n->g, (void *)n->Wk, (void *)n->WkT,
                    (void *)n->bias, (void *)n->wpart, (void *)n->lpart})
        if (p) (void)hipFree(p);
    delete n;
}

int64_t sci_wsnet_param_count(void) { return (int64_t)kNetLayers * kNetSlots; }

int sci_wsnet_set_loss(sci_ctx *ctx, sci_wsnet *n, int32_t kind)
{
    if (!ctx || !n) return SCI_ERR_INVALID_ARG;
    if (kind != SCI_WSNET_LOSS_DUAL && kind != SCI_WSNET_LOSS_THETA)
        return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: unknown loss kind");
    if (kind == SCI_WSNET_LOSS_THETA && n->c_out != 2)
        return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: the theta loss needs the two dual channels (c_out = 2)");
    n->loss = kind;
    return SCI_OK;
}

int sci_wsnet_set_params(sci_ctx *ctx, sci_wsnet *n, const float *host, int64_t count)
{
    if (!ctx || !n || !host || count != sci_wsnet_param_count())
        return ctx ? fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: set_params needs param_count floats") : SCI_ERR_INVALID_ARG;
    const size_t pb = (size_t)count * sizeof(float);
    hipError_t e;
    if ((e = hipMemcpy(n->w, host, pb, hipMemcpyHostToDevice)) != hipSuccess) return fail_hip(ctx, e, "hipMemcpy");
    if ((e = hipMemset(n->m, 0, pb)) != hipSuccess || (e = hipMemset(n->v, 0, pb)) != hipSuccess)
        return fail_hip(ctx, e, "hipMemset");
    n->step = 0;
    adam(n, 0.0f, nullptr); // repack (zeroes entries outside the layers' channels)
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_hip(ctx, e, "wsnet repack");
    return SCI_OK;
}

int sci_wsnet_get_params(sci_ctx *ctx, sci_wsnet *n, float *host, int64_t count)
{
    if (!ctx || !n || !host || count != sci_wsnet_param_count())
        return ctx ? fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: get_params needs param_count floats") : SCI_ERR_INVALID_ARG;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host, n->w, (size_t)count * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? SCI_OK : fail_hip(ctx, e, "hipMemcpy");
}

int sci_wsnet_forward(sci_ctx *ctx, sci_wsnet *n, sci_dims d, const float *X, const float *P_base, float *Y_out,
                      int32_t tv, float *dual_out, hipStream_t stream)
{
    int st = check_net_args(ctx, n, d, X);
    if (st != SCI_OK) return st;
    if (dual_out && (tv < SCI_TV_ATV || tv > SCI_TV_VTV || n->c_out != 2))
        return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: dual output needs a known tv and c_out = 2");
    const size_t V = (size_t)d.nx * d.ny * d.B;
    if ((st = ensure_acts(ctx, n, V, stream)) != SCI_OK) return st;
    const float *base = n->c_in == 3 ? P_base : nullptr;
    // ATV and ITV2D project pointwise: the last layer writes the dual itself
    const bool fused = dual_out && !Y_out && tv != SCI_TV_VTV;
    forward(n, d, X, base, false, fused ? dual_out : nullptr, tv, stream);
    if (Y_out) launch_copy(n->y, Y_out, V * (size_t)n->c_out * sizeof(float), stream);
    if (dual_out && !fused) wsnet_dual_from_net(d.nx, d.ny, d.B, tv, n->y, base, dual_out, stream);
    return check_launch(ctx, "wsnet forward");
}

int sci_wsnet_grads(sci_ctx *ctx, sci_wsnet *n, sci_dims d, const float *X, const float *P_base, const float *target,
                    float *grad_host, double *loss_host, hipStream_t stream)
{
    int st = check_net_args(ctx, n, d, X);
    if (st != SCI_OK) return st;
    if (!target) return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: null target");
    const size_t V = (size_t)d.nx * d.ny * d.B;
    if ((st = ensure_acts(ctx, n, V, stream)) != SCI_OK) return st;
    forward(n, d, X, P_base, true, nullptr, 0, stream);
    backward(ctx, n, d, X, P_base, target, stream);
    if ((st = check_launch(ctx, "wsnet grads")) != SCI_OK) return st;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
    if (grad_host &&
        (e = hipMemcpy(grad_host, n->g, (size_t)kNetLayers * kNetSlots * sizeof(float), hipMemcpyDeviceToHost)) !=
            hipSuccess)
        return fail_hip(ctx, e, "hipMemcpy");
    if (loss_host) {
        double se = 0.0;
        if ((e = hipMemcpy(&se, n->lpart + wsnet_reduce_blocks(), sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
            return fail_hip(ctx, e, "hipMemcpy");
        *loss_host = loss_value(n, se, V);
    }
    return SCI_OK;
}

int sci_wsnet_train_step(sci_ctx *ctx, sci_wsnet *n, sci_dims d, const float *X, const float *P_base,
                         const float *target, float lr, double *loss_host, hipStream_t stream)
{
    int st = check_net_args(ctx, n, d, X);
    if (st != SCI_OK) return st;
    if (!target || !std::isfinite(lr) || lr < 0.0f) return fail(ctx, SCI_ERR_INVALID_ARG, "wsnet: bad target or lr");
    const size_t V = (size_t)d.nx * d.ny * d.B;
    if ((st = ensure_acts(ctx, n, V, stream)) != SCI_OK) return st;
    forward(n, d, X, P_base, true, nullptr, 0, stream);
    backward(ctx, n, d, X, P_base, target, stream);
    ++n->step;
    adam(n, lr, stream);
    if ((st = check_launch(ctx, "wsnet train step")) != SCI_OK) return st;
    if (loss_host) {
        double se = 0.0;
        hipError_t e = hipMemcpyAsync(ctx->host_scalars, n->lpart + wsnet_reduce_blocks(), sizeof(double),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail_hip(ctx, e, "loss readback");
        se = ctx->host_scalars[0];
        *loss_host = loss_value(n, se, V);
    }
    return SCI_OK;
}

} // extern "C"
