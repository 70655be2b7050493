// ATV-Clip denoiser iteration (Sec. 2.3; Algorithm 1, Clip box): iterative
// clipping with one dual field per difference direction,
//   theta_h = x - D_h^T w_h,  w_h <- clip(w_h + D_h theta_h / alpha, T)
// and the same along the vertical direction, T = 2 lambda. The two
// directions never interact. One pass over HBM per iteration: a thread owns
// one voxel and reads its row / column neighbours (x and w at j-1, j, j+1
// and i-1, i, i+1; the neighbours are served by the caches).
#include <hip/hip_runtime.h>

#include "sci_internal.h"

namespace sci {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_clip(int nx, int ny, uint32_t V, const float *__restrict__ x,
                                                 const float *__restrict__ w, float *__restrict__ wn,
                                                 float inv_alpha, float T)
{
    const uint32_t o = blockIdx.x * kBlock + threadIdx.x;
    if (o >= V) return;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t r = o % plane;
    const int i = (int)(r / (uint32_t)ny), j = (int)(r % (uint32_t)ny);
    float nh = 0.0f, nv = 0.0f; // no difference at j = ny-1 (h) / i = nx-1 (v): the dual stays 0
    if (j < ny - 1) {
        const float *wh = w;
        const float wm = (w && j >= 1) ? wh[o - 1] : 0.0f;
        const float w0 = w ? wh[o] : 0.0f;
        const float wp = (w && j + 1 < ny - 1) ? wh[o + 1] : 0.0f;
        const float t0 = x[o] - (wm - w0);     // theta_h at j
        const float t1 = x[o + 1] - (w0 - wp); // theta_h at j+1
        nh = fminf(fmaxf(fmaf(t1 - t0, inv_alpha, w0), -T), T);
    }
    if (i < nx - 1) {
        const float *wv = w ? w + V : nullptr;
        const float wm = (wv && i >= 1) ? wv[o - ny] : 0.0f;
        const float w0 = wv ? wv[o] : 0.0f;
        const float wp = (wv && i + 1 < nx - 1) ? wv[o + ny] : 0.0f;
        const float t0 = x[o] - (wm - w0);
        const float t1 = x[o + ny] - (w0 - wp);
        nv = fminf(fmaxf(fmaf(t1 - t0, inv_alpha, w0), -T), T);
    }
    wn[o] = nh;
    wn[V + o] = nv;
}

} // namespace

void launch_clip(int nx, int ny, int B, const float *x, const float *w, float *w_next, float alpha, float lambda,
                 hipStream_t s)
{
    const uint32_t V = (uint32_t)nx * (uint32_t)ny * (uint32_t)B;
    hipLaunchKernelGGL(k_clip, dim3((V + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nx, ny, V, x, w, w_next,
                       1.0f / alpha, 2.0f * lambda);
}

} // namespace sci
