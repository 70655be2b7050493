// Sensing-operator kernels: Phi (Eq. (3)-(4)), Phi^T, the diagonal of
// Phi Phi^T, and the element-wise GAP / ADMM projections (Eq. (21), Eq. (24)).
//
// All of them are HBM streams over [B][nx][ny] volumes: one thread per pixel
// (i, j), consecutive threads on consecutive columns (coalesced), looping
// over the B frames. The per-pixel sum over frames stays in a register.
#include <hip/hip_runtime.h>

#include "sci_internal.h"

namespace sci {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(size_t n)
{
    size_t g = (n + kBlock - 1) / kBlock;
    return (unsigned)(g > 0 ? g : 1);
}

__global__ __launch_bounds__(kBlock) void k_forward(uint32_t npix, int B, const float *__restrict__ C,
                                                    const float *__restrict__ X, float *__restrict__ Y)
{
    uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    float acc = 0.0f;
    for (int k = 0; k < B; ++k) {
        uint32_t o = (uint32_t)k * npix + pix;
        acc = fmaf(C[o], X[o], acc);
    }
    Y[pix] = acc;
}

__global__ __launch_bounds__(kBlock) void k_adjoint(uint32_t npix, int B, const float *__restrict__ C,
                                                    const float *__restrict__ Y, float *__restrict__ X)
{
    uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    float y = Y[pix];
    for (int k = 0; k < B; ++k) {
        uint32_t o = (uint32_t)k * npix + pix;
        X[o] = C[o] * y;
    }
}

__global__ __launch_bounds__(kBlock) void k_weights(uint32_t npix, int B, const float *__restrict__ C, float rho,
                                                    float *__restrict__ Sinv)
{
    uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    float s = 0.0f;
    for (int k = 0; k < B; ++k) {
        float c = C[(uint32_t)k * npix + pix];
        s = fmaf(c, c, s);
    }
    s = s + rho;
    Sinv[pix] = s > 0.0f ? 1.0f / s : 0.0f;
}

// Projection modes: what the kernels take as v, the point they project.
//   kProjGap    v = theta (Eq. (21))
//   kProjAdmm   v = theta - u (Eq. (24)); the kernel also writes the denoiser
//               input s = u + x, and x only when x is non-null
//   kProjFista  v = theta + ex (theta - u), FISTA's extrapolated point formed
//               on load from the newest iterate (theta) and the one before (u),
//               the same expression as k_extrapolate (Sec. 2.2)
//   kProjTwist  v = a2 w + a1 theta + ex u, TwIST's two-step update from the
//               denoised point (w), the newest iterate (theta) and the one
//               before (u), the same expression as k_two_step (Sec. 2.2); the
//               kernel also stores v, the new iterate, to svol
constexpr int kProjGap = 0, kProjAdmm = 1, kProjFista = 2, kProjTwist = 3;

__device__ inline float fista_point(float x, float xp, float ex) { return fmaf(ex, x - xp, x); }
__device__ inline float twist_point(float xp, float x, float th, float a0, float a1, float a2)
{
    return fmaf(a2, th, fmaf(a1, x, a0 * xp));
}

// x_k = v_k + C_k r with r = (Y - sum_k C_k v_k) Sinv.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_project(uint32_t npix, int B, float ex, float a1, float a2, const float *__restrict__ w, const float *__restrict__ theta,
                                                    const float *__restrict__ u, const float *__restrict__ C,
                                                    const float *__restrict__ Y, const float *__restrict__ Sinv,
                                                    float *__restrict__ x, float *__restrict__ svol)
{
    uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    constexpr bool ADMM = MODE == kProjAdmm;
    float acc = 0.0f;
    for (int k = 0; k < B; ++k) {
        uint32_t o = (uint32_t)k * npix + pix;
        float v = MODE == kProjGap    ? theta[o]
                : ADMM                ? theta[o] - u[o]
                : MODE == kProjFista ? fista_point(theta[o], u[o], ex)
                                     : twist_point(u[o], theta[o], w[o], ex, a1, a2);
        acc = fmaf(C[o], v, acc);
    }
    float r = (Y[pix] - acc) * Sinv[pix];
    for (int k = 0; k < B; ++k) {
        uint32_t o = (uint32_t)k * npix + pix;
        float v = MODE == kProjGap    ? theta[o]
                : ADMM                ? theta[o] - u[o]
                : MODE == kProjFista ? fista_point(theta[o], u[o], ex)
                                     : twist_point(u[o], theta[o], w[o], ex, a1, a2);
        float xv = fmaf(C[o], r, v);
        if (!ADMM || x) x[o] = xv;
        if (ADMM) svol[o] = u[o] + xv;
        if (MODE == kProjTwist) svol[o] = v;
    }
}

// Same projection with every frame of the pixel held in registers (KB >= B),
// so theta, u and C are read from memory once.
template <int MODE, int KB>
__global__ __launch_bounds__(kBlock) void k_project_reg(uint32_t npix, int B, float ex, float a1, float a2, const float *__restrict__ w, const float *__restrict__ theta,
                                                        const float *__restrict__ u, const float *__restrict__ C,
                                                        const float *__restrict__ Y, const float *__restrict__ Sinv,
                                                        float *__restrict__ x, float *__restrict__ svol)
{
    uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    constexpr bool ADMM = MODE == kProjAdmm;
    float v[KB], c[KB], uu[KB];
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * npix + pix;
            c[k] = C[o];
            if (ADMM) {
                uu[k] = u[o];
                v[k] = theta[o] - uu[k];
            } else if (MODE == kProjFista) {
                v[k] = fista_point(theta[o], u[o], ex);
            } else if (MODE == kProjTwist) {
                v[k] = twist_point(u[o], theta[o], w[o], ex, a1, a2);
            } else {
                v[k] = theta[o];
            }
            acc = fmaf(c[k], v[k], acc);
        }
    }
    const float r = (Y[pix] - acc) * Sinv[pix];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * npix + pix;
            const float xv = fmaf(c[k], r, v[k]);
            if (!ADMM || x) x[o] = xv;
            if (ADMM) svol[o] = uu[k] + xv;
            if (MODE == kProjTwist) svol[o] = v[k];
        }
    }
}

// Two adjacent pixels per thread (8-byte loads and stores), every frame in
// registers; the same per-pixel arithmetic as k_project_reg.
template <int MODE, int KB>
__global__ __launch_bounds__(kBlock) void k_project_reg2(uint32_t npair, uint32_t npix, int B, float ex, float a1, float a2, const float2 *__restrict__ w,
                                                         const float2 *__restrict__ theta,
                                                         const float2 *__restrict__ u, const float2 *__restrict__ C,
                                                         const float2 *__restrict__ Y,
                                                         const float2 *__restrict__ Sinv, float2 *__restrict__ x,
                                                         float2 *__restrict__ svol)
{
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= npair) return;
    constexpr bool ADMM = MODE == kProjAdmm;
    const uint32_t fstride = npix / 2; // float2 elements per frame
    float2 v[KB], c[KB], uu[KB];
    float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * fstride + q;
            c[k] = C[o];
            if (ADMM) {
                uu[k] = u[o];
                const float2 t = theta[o];
                v[k] = make_float2(t.x - uu[k].x, t.y - uu[k].y);
            } else if (MODE == kProjFista) {
                const float2 t = theta[o], tp = u[o];
                v[k] = make_float2(fista_point(t.x, tp.x, ex), fista_point(t.y, tp.y, ex));
            } else if (MODE == kProjTwist) {
                const float2 t = theta[o], tp = u[o], tw = w[o];
                v[k] = make_float2(twist_point(tp.x, t.x, tw.x, ex, a1, a2), twist_point(tp.y, t.y, tw.y, ex, a1, a2));
            } else {
                v[k] = theta[o];
            }
            acc0 = fmaf(c[k].x, v[k].x, acc0);
            acc1 = fmaf(c[k].y, v[k].y, acc1);
        }
    }
    const float2 yv = Y[q], sv = Sinv[q];
    const float r0 = (yv.x - acc0) * sv.x, r1 = (yv.y - acc1) * sv.y;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * fstride + q;
            const float2 xv = make_float2(fmaf(c[k].x, r0, v[k].x), fmaf(c[k].y, r1, v[k].y));
            if (!ADMM || x) x[o] = xv;
            if (ADMM) svol[o] = make_float2(uu[k].x + xv.x, uu[k].y + xv.y);
            if (MODE == kProjTwist) svol[o] = v[k];
        }
    }
}

// Binary masks packed one bit per frame into a 32-bit word per pixel
// (B <= 32): bits[pix] bit k = (C_k(pix) == 1). flag (set to 1 beforehand)
// is cleared when any entry is neither 0 nor 1; the projection then reads C.
__global__ __launch_bounds__(kBlock) void k_pack_masks(uint32_t npix, int B, const float *__restrict__ C,
                                                       uint32_t *__restrict__ bits, int *__restrict__ flag)
{
    const uint32_t pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= npix) return;
    uint32_t b = 0u;
    bool ok = true;
    for (int k = 0; k < B; ++k) {
        const float c = C[(uint32_t)k * npix + pix];
        if (c == 1.0f) b |= 1u << k;
        else if (c != 0.0f) ok = false;
    }
    bits[pix] = b;
    if (!ok) atomicAnd(flag, 0);
}

__global__ void k_set_flag(int *flag, int v) { *flag = v; }

// The projection with binary masks read from the packed bits: C_k is 0 or
// 1, so fmaf(C_k, v, acc) and fmaf(C_k, r, v) reduce exactly to a select of
// acc + v / acc and v + r / v, the same values the float path produces. Two
// adjacent pixels per thread; when *flag is 0 the float masks are used.
template <int MODE, int KB>
__global__ __launch_bounds__(kBlock) void k_project_bits(uint32_t npair, uint32_t npix, int B, float ex, float a1, float a2, const float2 *__restrict__ w,
                                                         const float2 *__restrict__ theta,
                                                         const float2 *__restrict__ u, const float2 *__restrict__ C,
                                                         const uint2 *__restrict__ bits, const int *__restrict__ flag,
                                                         const float2 *__restrict__ Y, const float2 *__restrict__ Sinv,
                                                         float2 *__restrict__ x, float2 *__restrict__ svol)
{
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= npair) return;
    constexpr bool ADMM = MODE == kProjAdmm;
    const uint32_t fstride = npix / 2;
    const bool packed = *flag != 0;
    float2 v[KB], uu[KB];
    uint2 m = packed ? bits[q] : make_uint2(0u, 0u);
    float2 c[KB];
    float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * fstride + q;
            if (packed) c[k] = make_float2((m.x >> k) & 1u ? 1.0f : 0.0f, (m.y >> k) & 1u ? 1.0f : 0.0f);
            else c[k] = C[o];
            if (ADMM) {
                uu[k] = u[o];
                const float2 t = theta[o];
                v[k] = make_float2(t.x - uu[k].x, t.y - uu[k].y);
            } else if (MODE == kProjFista) {
                const float2 t = theta[o], tp = u[o];
                v[k] = make_float2(fista_point(t.x, tp.x, ex), fista_point(t.y, tp.y, ex));
            } else if (MODE == kProjTwist) {
                const float2 t = theta[o], tp = u[o], tw = w[o];
                v[k] = make_float2(twist_point(tp.x, t.x, tw.x, ex, a1, a2), twist_point(tp.y, t.y, tw.y, ex, a1, a2));
            } else {
                v[k] = theta[o];
            }
            acc0 = fmaf(c[k].x, v[k].x, acc0);
            acc1 = fmaf(c[k].y, v[k].y, acc1);
        }
    }
    const float2 yv = Y[q], sv = Sinv[q];
    const float r0 = (yv.x - acc0) * sv.x, r1 = (yv.y - acc1) * sv.y;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * fstride + q;
            const float2 xv = make_float2(fmaf(c[k].x, r0, v[k].x), fmaf(c[k].y, r1, v[k].y));
            if (!ADMM || x) x[o] = xv;
            if (ADMM) svol[o] = make_float2(uu[k].x + xv.x, uu[k].y + xv.y);
            if (MODE == kProjTwist) svol[o] = v[k];
        }
    }
}

template <int MODE>
void launch_project(uint32_t npix, int B, float ex, const float *theta, const float *u, const float *C,
                    const float *Y, const float *Sinv, float *x, float *svol, hipStream_t s,
                    const uint32_t *cbits = nullptr, const int *cflag = nullptr, float a1 = 0.0f, float a2 = 0.0f,
                    const float *w = nullptr)
{
    const dim3 g(grid_for(npix)), b(kBlock);
    auto al8 = [](const void *p) { return p == nullptr || ((uintptr_t)p & 7u) == 0; };
    if (npix % 2 == 0 && B <= 32 && al8(theta) && al8(u) && al8(C) && al8(Y) && al8(Sinv) && al8(x) && al8(svol) && al8(w)) {
        const uint32_t npair = npix / 2;
        const dim3 g2(grid_for(npair));
        const float2 *t2 = (const float2 *)theta, *u2 = (const float2 *)u, *C2 = (const float2 *)C;
        const float2 *Y2 = (const float2 *)Y, *S2 = (const float2 *)Sinv;
        float2 *x2 = (float2 *)x, *s2 = (float2 *)svol;
        if (cbits && cflag && al8(cbits)) {
            const uint2 *m2 = (const uint2 *)cbits;
            if (B <= 8) hipLaunchKernelGGL((k_project_bits<MODE, 8>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, m2, cflag, Y2, S2, x2, s2);
            else if (B <= 16) hipLaunchKernelGGL((k_project_bits<MODE, 16>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, m2, cflag, Y2, S2, x2, s2);
            else if (B <= 24) hipLaunchKernelGGL((k_project_bits<MODE, 24>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, m2, cflag, Y2, S2, x2, s2);
            else hipLaunchKernelGGL((k_project_bits<MODE, 32>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, m2, cflag, Y2, S2, x2, s2);
            return;
        }
        if (B <= 8) hipLaunchKernelGGL((k_project_reg2<MODE, 8>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, Y2, S2, x2, s2);
        else if (B <= 16) hipLaunchKernelGGL((k_project_reg2<MODE, 16>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, Y2, S2, x2, s2);
        else if (B <= 24) hipLaunchKernelGGL((k_project_reg2<MODE, 24>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, Y2, S2, x2, s2);
        else hipLaunchKernelGGL((k_project_reg2<MODE, 32>), g2, b, 0, s, npair, npix, B, ex, a1, a2, (const float2 *)w, t2, u2, C2, Y2, S2, x2, s2);
        return;
    }
    if (B <= 8) hipLaunchKernelGGL((k_project_reg<MODE, 8>), g, b, 0, s, npix, B, ex, a1, a2, w, theta, u, C, Y, Sinv, x, svol);
    else if (B <= 16) hipLaunchKernelGGL((k_project_reg<MODE, 16>), g, b, 0, s, npix, B, ex, a1, a2, w, theta, u, C, Y, Sinv, x, svol);
    else if (B <= 32) hipLaunchKernelGGL((k_project_reg<MODE, 32>), g, b, 0, s, npix, B, ex, a1, a2, w, theta, u, C, Y, Sinv, x, svol);
    else hipLaunchKernelGGL((k_project<MODE>), g, b, 0, s, npix, B, ex, a1, a2, w, theta, u, C, Y, Sinv, x, svol);
}

__global__ __launch_bounds__(kBlock) void k_copy4(uint32_t n4, const uint32_t *__restrict__ src,
                                                  uint32_t *__restrict__ dst)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_copy1(uint32_t n, const uint8_t *__restrict__ src,
                                                  uint8_t *__restrict__ dst)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_zero4(uint32_t n4, uint32_t *__restrict__ dst)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n4) dst[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_zero1(uint32_t n, uint8_t *__restrict__ dst)
{
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_fill(uint32_t n, float v, float *__restrict__ dst)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = v;
}

// FISTA extrapolation theta = x + c (x - x_prev).
__global__ __launch_bounds__(kBlock) void k_extrapolate(uint32_t n, float c, const float *__restrict__ x,
                                                        const float *__restrict__ xp, float *__restrict__ th)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float xv = x[i];
    th[i] = fmaf(c, xv - xp[i], xv);
}

// TwIST two-step update out = a0 x_prev + a1 x + a2 theta.
__global__ __launch_bounds__(kBlock) void k_two_step(uint32_t n, float a0, float a1, float a2,
                                                     const float *__restrict__ xp, const float *__restrict__ x,
                                                     const float *__restrict__ th, float *__restrict__ out)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = fmaf(a2, th[i], fmaf(a1, x[i], a0 * xp[i]));
}

} // namespace

void launch_fill(float *dst, float v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, (uint32_t)n, v, dst);
}

void launch_extrapolate(size_t n, float c, const float *x, const float *xp, float *th, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_extrapolate, dim3(grid_for(n)), dim3(kBlock), 0, s, (uint32_t)n, c, x, xp, th);
}

void launch_two_step(size_t n, float a0, float a1, float a2, const float *xp, const float *x, const float *th,
                     float *out, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_two_step, dim3(grid_for(n)), dim3(kBlock), 0, s, (uint32_t)n, a0, a1, a2, xp, x, th, out);
}

void launch_forward(int nx, int ny, int B, const float *C, const float *X, float *Y, hipStream_t s)
{
    uint32_t npix = (uint32_t)nx * (uint32_t)ny;
    hipLaunchKernelGGL(k_forward, dim3(grid_for(npix)), dim3(kBlock), 0, s, npix, B, C, X, Y);
}

void launch_adjoint(int nx, int ny, int B, const float *C, const float *Y, float *X, hipStream_t s)
{
    uint32_t npix = (uint32_t)nx * (uint32_t)ny;
    hipLaunchKernelGGL(k_adjoint, dim3(grid_for(npix)), dim3(kBlock), 0, s, npix, B, C, Y, X);
}

void launch_weights(int nx, int ny, int B, const float *C, float rho, float *Sinv, hipStream_t s)
{
    uint32_t npix = (uint32_t)nx * (uint32_t)ny;
    hipLaunchKernelGGL(k_weights, dim3(grid_for(npix)), dim3(kBlock), 0, s, npix, B, C, rho, Sinv);
}

void launch_gap_project(int nx, int ny, int B, const float *theta, const float *C, const float *Y,
                        const float *Sinv, float *x, hipStream_t s, const uint32_t *cbits, const int *cflag)
{
    launch_project<kProjGap>((uint32_t)nx * (uint32_t)ny, B, 0.0f, theta, nullptr, C, Y, Sinv, x, nullptr, s, cbits,
                             cflag);
}

void launch_admm_project(int nx, int ny, int B, const float *theta, const float *u, const float *C,
                         const float *Y, const float *Sinv, float *x, float *svol, hipStream_t s,
                         const uint32_t *cbits, const int *cflag)
{
    launch_project<kProjAdmm>((uint32_t)nx * (uint32_t)ny, B, 0.0f, theta, u, C, Y, Sinv, x, svol, s, cbits, cflag);
}

void launch_fista_project(int nx, int ny, int B, const float *x, const float *x_prev, float ex, const float *C,
                          const float *Y, const float *W, float *z, hipStream_t s, const uint32_t *cbits,
                          const int *cflag)
{
    launch_project<kProjFista>((uint32_t)nx * (uint32_t)ny, B, ex, x, x_prev, C, Y, W, z, nullptr, s, cbits, cflag);
}

void launch_twist_project(int nx, int ny, int B, const float *x, const float *x_prev, const float *theta, float a0,
                          float a1, float a2, const float *C, const float *Y, const float *W, float *z, float *x_next,
                          hipStream_t s, const uint32_t *cbits, const int *cflag)
{
    launch_project<kProjTwist>((uint32_t)nx * (uint32_t)ny, B, a0, x, x_prev, C, Y, W, z, x_next, s, cbits, cflag, a1,
                               a2, theta);
}

void launch_pack_masks(int nx, int ny, int B, const float *C, uint32_t *bits, int *flag, hipStream_t s)
{
    const uint32_t npix = (uint32_t)nx * (uint32_t)ny;
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, s, flag, B <= 32 ? 1 : 0);
    if (B <= 32) hipLaunchKernelGGL(k_pack_masks, dim3(grid_for(npix)), dim3(kBlock), 0, s, npix, B, C, bits, flag);
}

// Device-to-device copy and zero fill as plain kernels, so that they can be
// captured into HIP graphs (no memset / memcpy nodes).
void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if ((bytes & 3) == 0 && ((uintptr_t)src & 3) == 0 && ((uintptr_t)dst & 3) == 0) {
        uint32_t n4 = (uint32_t)(bytes / 4);
        hipLaunchKernelGGL(k_copy4, dim3(grid_for(n4)), dim3(kBlock), 0, s, n4, (const uint32_t *)src,
                           (uint32_t *)dst);
    } else {
        hipLaunchKernelGGL(k_copy1, dim3(grid_for(bytes)), dim3(kBlock), 0, s, (uint32_t)bytes,
                           (const uint8_t *)src, (uint8_t *)dst);
    }
}

void launch_zero(void *dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if ((bytes & 3) == 0 && ((uintptr_t)dst & 3) == 0) {
        uint32_t n4 = (uint32_t)(bytes / 4);
        hipLaunchKernelGGL(k_zero4, dim3(grid_for(n4)), dim3(kBlock), 0, s, n4, (uint32_t *)dst);
    } else {
        hipLaunchKernelGGL(k_zero1, dim3(grid_for(bytes)), dim3(kBlock), 0, s, (uint32_t)bytes, (uint8_t *)dst);
    }
}

} // namespace sci
