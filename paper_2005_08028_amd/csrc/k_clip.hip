// ATV-Clip denoiser iteration (Sec. 2.3; Algorithm 1, Clip box): iterative
// clipping with one dual field per difference direction,
//   theta_h = x - D_h^T w_h,  w_h <- clip(w_h + D_h theta_h / alpha, T)
// and the same along the vertical direction, T = 2 lambda. The two
// directions never interact. One pass over HBM per iteration: a thread owns
// one column of a frame, every gridDim.y-th row of it, and reads the row /
// column neighbours (x and w at j-1, j, j+1 and i-1, i, i+1) through the
// caches. The duals are stored in any of the dual types (arithmetic in
// float32; 16-bit values rounded to nearest even where they are stored).
#include <hip/hip_runtime.h>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

constexpr int kBlock = 256;

template <int DT>
__global__ __launch_bounds__(kBlock) void k_clip(int nx, int ny, int B, const float *__restrict__ x,
                                                 const typename Dual<DT>::T *__restrict__ w,
                                                 typename Dual<DT>::T *__restrict__ wn, float inv_alpha, float T)
{
    using D = Dual<DT>;
    const int j = (int)blockIdx.x * kBlock + (int)threadIdx.x;
    if (j >= ny) return;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const uint32_t fo = (uint32_t)blockIdx.z * plane;
    for (int i = (int)blockIdx.y; i < nx; i += (int)gridDim.y) {
        const uint32_t o = fo + (uint32_t)i * ny + (uint32_t)j;
        const bool hd = j < ny - 1, vd = i < nx - 1; // a difference exists at this voxel
        // loads from in-bounds addresses (o stands in for a missing neighbour), masked afterwards
        const uint32_t oR = hd ? o + 1 : o, oD = vd ? o + ny : o;
        const float x0 = x[o], xr = x[oR], xd = x[oD];
        float hm = 0.0f, h0 = 0.0f, hp = 0.0f, vm = 0.0f, v0 = 0.0f, vp = 0.0f;
        if (w) {
            hm = D::ld(w, j >= 1 ? o - 1 : o);
            h0 = D::ld(w, o);
            hp = D::ld(w, oR);
            vm = D::ld(w, V + (i >= 1 ? o - ny : o));
            v0 = D::ld(w, V + o);
            vp = D::ld(w, V + oD);
        }
        float nh = 0.0f, nv = 0.0f; // no difference at j = ny-1 (h) / i = nx-1 (v): the dual stays 0
        if (hd) {
            const float wm = j >= 1 ? hm : 0.0f, wp = j + 1 < ny - 1 ? hp : 0.0f;
            const float t0 = x0 - (wm - h0); // theta_h at j
            const float t1 = xr - (h0 - wp); // theta_h at j+1
            nh = fminf(fmaxf(fmaf(t1 - t0, inv_alpha, h0), -T), T);
        }
        if (vd) {
            const float wm = i >= 1 ? vm : 0.0f, wp = i + 1 < nx - 1 ? vp : 0.0f;
            const float t0 = x0 - (wm - v0);
            const float t1 = xd - (v0 - wp);
            nv = fminf(fmaxf(fmaf(t1 - t0, inv_alpha, v0), -T), T);
        }
        D::st(wn, o, nh);
        D::st(wn, V + o, nv);
    }
}

} // namespace

int launch_clip(int dual_dtype, int nx, int ny, int B, const float *x, const void *w, void *w_next, float alpha,
                float lambda, hipStream_t s)
{
    const dim3 grid((ny + kBlock - 1) / kBlock, (unsigned)(nx < 65535 ? nx : 65535), (unsigned)B);
    const float ia = 1.0f / alpha, T = 2.0f * lambda;
    switch (dual_dtype) {
    case DT_F32:
        hipLaunchKernelGGL(k_clip<DT_F32>, grid, dim3(kBlock), 0, s, nx, ny, B, x, (const float *)w, (float *)w_next,
                           ia, T);
        return SCI_OK;
    case DT_BF16:
        hipLaunchKernelGGL(k_clip<DT_BF16>, grid, dim3(kBlock), 0, s, nx, ny, B, x, (const uint16_t *)w,
                           (uint16_t *)w_next, ia, T);
        return SCI_OK;
    case DT_F16:
        hipLaunchKernelGGL(k_clip<DT_F16>, grid, dim3(kBlock), 0, s, nx, ny, B, x, (const _Float16 *)w,
                           (_Float16 *)w_next, ia, T);
        return SCI_OK;
    }
    return SCI_ERR_UNSUPPORTED;
}

} // namespace sci
