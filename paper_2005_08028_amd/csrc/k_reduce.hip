// FP64 reductions on the GPU: squared differences (PSNR), the measurement
// residual ||Y - Phi X||^2, and the terms of the denoiser's duality gap.
//
// Deterministic two-stage scheme: a fixed grid of kRedBlocks workgroups,
// each thread accumulates a grid-stride slice in double, the workgroup folds
// its 256 values by a fixed LDS tree into one partial; a single workgroup
// then folds the partials in the same fixed order. No floating-point
// atomics, so repeated calls return bit-identical results.
#include <hip/hip_runtime.h>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// Fold 256 doubles held one per thread; result valid in thread 0.
__device__ inline double block_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    double r = lds[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kRedThreads) void k_sqdiff_part(int64_t n, const float *__restrict__ a,
                                                             const float *__restrict__ b,
                                                             double *__restrict__ part)
{
    __shared__ double lds[kRedThreads];
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; c < n; c += (int64_t)kRedBlocks * kRedThreads) {
        const double d = (double)a[c] - (double)b[c];
        acc += d * d;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_resid_part(int nx, int ny, int B, const float *__restrict__ C,
                                                            const float *__restrict__ X,
                                                            const float *__restrict__ Y, double *__restrict__ part)
{
    __shared__ double lds[kRedThreads];
    const int64_t npix = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; c < npix;
         c += (int64_t)kRedBlocks * kRedThreads) {
        double f = 0.0;
        for (int k = 0; k < B; ++k) f += (double)C[k * npix + c] * (double)X[k * npix + c];
        const double d = (double)Y[c] - f;
        acc += d * d;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// theta = x - lambda D^T p at voxel (k, i, j), in double.
template <int DT>
__device__ inline double theta64(int nx, int ny, uint32_t V, const float *x, const typename Dual<DT>::T *p,
                                 double lam, uint32_t fo, int i, int j)
{
    using D = Dual<DT>;
    const uint32_t o = fo + (uint32_t)i * ny + j;
    double a = 0.0;
    if (j >= 1) a += (double)D::ld(p, o - 1);
    if (j + 1 < ny) a -= (double)D::ld(p, o);
    if (i >= 1) a += (double)D::ld(p, V + o - ny);
    if (i + 1 < nx) a -= (double)D::ld(p, V + o);
    return (double)x[o] - lam * a;
}

// Partials [3][kRedBlocks]: TV(theta), <D theta, p>, ||theta - x||^2. One
// thread per pixel, looping over frames (VTV needs the per-pixel norm over
// all frames).
template <int TV, int DT>
__global__ __launch_bounds__(kRedThreads) void k_gap_part(int nx, int ny, int B, double lam,
                                                          const float *__restrict__ x,
                                                          const typename Dual<DT>::T *__restrict__ p,
                                                          double *__restrict__ part)
{
    using D = Dual<DT>;
    __shared__ double lds[kRedThreads];
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    double tv = 0.0, inner = 0.0, fid = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; c < (int64_t)plane;
         c += (int64_t)kRedBlocks * kRedThreads) {
        const int i = (int)(c / ny), j = (int)(c % ny);
        double s2 = 0.0;
        for (int k = 0; k < B; ++k) {
            const uint32_t fo = (uint32_t)k * plane;
            const uint32_t o = fo + (uint32_t)c;
            const double th = theta64<DT>(nx, ny, V, x, p, lam, fo, i, j);
            const double gh = (j + 1 < ny) ? theta64<DT>(nx, ny, V, x, p, lam, fo, i, j + 1) - th : 0.0;
            const double gv = (i + 1 < nx) ? theta64<DT>(nx, ny, V, x, p, lam, fo, i + 1, j) - th : 0.0;
            const double ph = (j + 1 < ny) ? (double)D::ld(p, o) : 0.0;
            const double pv = (i + 1 < nx) ? (double)D::ld(p, V + o) : 0.0;
            inner += gh * ph + gv * pv;
            const double dx = th - (double)x[o];
            fid += dx * dx;
            if (TV == TV_ATV) tv += fabs(gh) + fabs(gv);
            else if (TV == TV_ITV2D) tv += sqrt(gh * gh + gv * gv);
            else s2 += gh * gh + gv * gv;
        }
        if (TV == TV_VTV) tv += sqrt(s2);
    }
    double r = block_sum(tv, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
    r = block_sum(inner, lds);
    if (threadIdx.x == 0) part[kRedBlocks + blockIdx.x] = r;
    r = block_sum(fid, lds);
    if (threadIdx.x == 0) part[2 * kRedBlocks + blockIdx.x] = r;
}

// out[c] = sum of part[c * kRedBlocks .. + kRedBlocks) in a fixed order.
__global__ __launch_bounds__(kRedThreads) void k_final(int nch, const double *__restrict__ part,
                                                       double *__restrict__ out)
{
    __shared__ double lds[kRedThreads];
    for (int c = 0; c < nch; ++c) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads) acc += part[c * kRedBlocks + b];
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) out[c] = s;
    }
}

// Largest S_ij = sum_k C_kij^2 (accumulated as in the weights kernel): one
// maximum per workgroup, then one workgroup takes the maximum of those.
__device__ inline float block_max(float v, float *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] = fmaxf(lds[threadIdx.x], lds[threadIdx.x + w]);
        __syncthreads();
    }
    float r = lds[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kRedThreads) void k_max_s_part(int nx, int ny, int B, const float *__restrict__ C,
                                                            float *__restrict__ part)
{
    __shared__ float lds[kRedThreads];
    const int64_t npix = (int64_t)nx * ny;
    float m = 0.0f;
    for (int64_t c = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; c < npix;
         c += (int64_t)kRedBlocks * kRedThreads) {
        float s = 0.0f;
        for (int k = 0; k < B; ++k) {
            const float v = C[k * npix + c];
            s = fmaf(v, v, s);
        }
        m = fmaxf(m, s);
    }
    const float r = block_max(m, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kRedThreads) void k_max_final(const float *__restrict__ part, double *__restrict__ out)
{
    __shared__ float lds[kRedThreads];
    float m = 0.0f;
    for (int b = threadIdx.x; b < kRedBlocks; b += kRedThreads) m = fmaxf(m, part[b]);
    const float r = block_max(m, lds);
    if (threadIdx.x == 0) out[0] = (double)r;
}

template <int TV>
void gap_tv_dt(int dual_dtype, int nx, int ny, int B, double lam, const float *x, const void *p, double *part,
               hipStream_t s)
{
    switch (dual_dtype) {
    case DT_F32:
        hipLaunchKernelGGL((k_gap_part<TV, DT_F32>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, nx, ny, B, lam, x,
                           (const float *)p, part);
        break;
    case DT_BF16:
        hipLaunchKernelGGL((k_gap_part<TV, DT_BF16>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, nx, ny, B, lam, x,
                           (const uint16_t *)p, part);
        break;
    default:
        hipLaunchKernelGGL((k_gap_part<TV, DT_F16>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, nx, ny, B, lam, x,
                           (const _Float16 *)p, part);
        break;
    }
}

} // namespace

int reduce_partial_blocks() { return kRedBlocks; }

void launch_sqdiff(int64_t n, const float *a, const float *b, double *partials, double *out_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqdiff_part, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, a, b, partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, 1, (const double *)partials, out_dev);
}

void launch_residual_sq(int nx, int ny, int B, const float *C, const float *X, const float *Y, double *partials,
                        double *out_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_resid_part, dim3(kRedBlocks), dim3(kRedThreads), 0, s, nx, ny, B, C, X, Y, partials);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, 1, (const double *)partials, out_dev);
}

void launch_max_s(int nx, int ny, int B, const float *C, double *partials, double *out_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_max_s_part, dim3(kRedBlocks), dim3(kRedThreads), 0, s, nx, ny, B, C, (float *)partials);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kRedThreads), 0, s, (const float *)partials, out_dev);
}

int launch_gap_terms(int tv, int dual_dtype, int nx, int ny, int B, float lam, const float *x, const void *p,
                     double *partials, double *out_dev, hipStream_t s)
{
    const double l = (double)lam;
    if (tv == TV_ATV) gap_tv_dt<TV_ATV>(dual_dtype, nx, ny, B, l, x, p, partials, s);
    else if (tv == TV_ITV2D) gap_tv_dt<TV_ITV2D>(dual_dtype, nx, ny, B, l, x, p, partials, s);
    else gap_tv_dt<TV_VTV>(dual_dtype, nx, ny, B, l, x, p, partials, s);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, s, 3, (const double *)partials, out_dev);
    return SCI_OK;
}

} // namespace sci
