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

// Gap terms of voxel o = (k, i, j): adds |D theta| (ATV, ITV2D) or
// |D theta|^2 (VTV, to s2), <D theta, p> and (theta - x)^2, all in double,
// with theta = x - lambda D^T p at (i, j), (i, j+1) and (i+1, j). Every load
// is issued unconditionally from an in-bounds address (o itself stands in
// for a missing neighbour) and masked afterwards, so a voxel's loads are in
// flight together instead of one branch at a time.
template <int TV, int DT>
__device__ __forceinline__ void gap_voxel(int nx, int ny, uint32_t V, const float *x, const typename Dual<DT>::T *p,
                                          double lam, uint32_t o, int i, int j, double &tv, double &inner,
                                          double &fid, double &s2)
{
    using D = Dual<DT>;
    const bool l = j >= 1, u = i >= 1, r = j + 1 < ny, dn = i + 1 < nx;
    const bool ru = r && u, dl = dn && l, r2 = j + 2 < ny, d2 = i + 2 < nx;
    const uint32_t oR = r ? o + 1 : o, oD = dn ? o + ny : o;
    // p_h at (i,j-1), (i,j), (i,j+1), (i+1,j-1), (i+1,j); p_v at (i-1,j), (i,j), (i-1,j+1), (i,j+1), (i+1,j)
    const float h_l = D::ld(p, l ? o - 1 : o), h_c = D::ld(p, o), h_r = D::ld(p, oR);
    const float h_dl = D::ld(p, dl ? oD - 1 : o), h_d = D::ld(p, oD);
    const float v_u = D::ld(p, V + (u ? o - ny : o)), v_c = D::ld(p, V + o);
    const float v_ur = D::ld(p, V + (ru ? oR - ny : o)), v_r = D::ld(p, V + oR), v_d = D::ld(p, V + oD);
    const float x_c = x[o], x_r = x[oR], x_d = x[oD];
    // theta = x - lambda ((p_h(j-1) - p_h(j)) + (p_v(i-1) - p_v(i))), terms without a difference are 0
    auto theta = [&](float xv, bool hl, float a, bool hc, float b, bool vu, float c, bool vc, float d) {
        double s = 0.0;
        s += hl ? (double)a : 0.0;
        s -= hc ? (double)b : 0.0;
        s += vu ? (double)c : 0.0;
        s -= vc ? (double)d : 0.0;
        return (double)xv - lam * s;
    };
    const double th = theta(x_c, l, h_l, r, h_c, u, v_u, dn, v_c);
    const double gh = r ? theta(x_r, true, h_c, r2, h_r, u, v_ur, dn, v_r) - th : 0.0;
    const double gv = dn ? theta(x_d, l, h_dl, r, h_d, true, v_c, d2, v_d) - th : 0.0;
    const double ph = r ? (double)h_c : 0.0;
    const double pv = dn ? (double)v_c : 0.0;
    inner += gh * ph + gv * pv;
    const double dx = th - (double)x_c;
    fid += dx * dx;
    if (TV == TV_ATV) tv += fabs(gh) + fabs(gv);
    else if (TV == TV_ITV2D) tv += sqrt(gh * gh + gv * gv);
    else s2 += gh * gh + gv * gv;
}

// Partials [3][kRedBlocks]: TV(theta), <D theta, p>, ||theta - x||^2. A
// workgroup covers kRedThreads consecutive columns (blockIdx.x) and every
// gridDim.y-th row (blockIdx.y); each thread walks its column through those
// rows and, per row, through all frames (VTV needs the per-pixel norm over
// them), four frames in flight. No integer division per voxel; neighbours
// come through the caches.
template <int TV, int DT>
__global__ __launch_bounds__(kRedThreads) void k_gap_part(int nx, int ny, int B, double lam,
                                                          const float *__restrict__ x,
                                                          const typename Dual<DT>::T *__restrict__ p,
                                                          double *__restrict__ part)
{
    __shared__ double lds[kRedThreads];
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int j = (int)blockIdx.x * kRedThreads + (int)threadIdx.x;
    double tv = 0.0, inner = 0.0, fid = 0.0;
    if (j < ny) {
        for (int i = (int)blockIdx.y; i < nx; i += (int)gridDim.y) {
            const uint32_t pix = (uint32_t)i * ny + (uint32_t)j;
            double s2 = 0.0;
#pragma unroll 4
            for (int k = 0; k < B; ++k)
                gap_voxel<TV, DT>(nx, ny, V, x, p, lam, (uint32_t)k * plane + pix, i, j, tv, inner, fid, s2);
            if (TV == TV_VTV) tv += sqrt(s2);
        }
    }
    const int b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int nb = (int)(gridDim.x * gridDim.y);
    double r = block_sum(tv, lds);
    if (threadIdx.x == 0) part[b] = r;
    r = block_sum(inner, lds);
    if (threadIdx.x == 0) part[nb + b] = r;
    r = block_sum(fid, lds);
    if (threadIdx.x == 0) part[2 * nb + b] = r;
}

// Grid of k_gap_part: column blocks x row strides, about kRedBlocks workgroups.
dim3 gap_grid(int nx, int ny)
{
    const int gx = (ny + kRedThreads - 1) / kRedThreads;
    int gy = kRedBlocks / gx;
    if (gy < 1) gy = 1;
    if (gy > nx) gy = nx;
    return dim3(gx, gy);
}

// out[c] = sum of part[c * n .. + n) in a fixed order (one workgroup).
__global__ __launch_bounds__(kRedThreads) void k_final_n(int nch, int n, const double *__restrict__ part,
                                                         double *__restrict__ out)
{
    __shared__ double lds[kRedThreads];
    for (int c = 0; c < nch; ++c) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < n; b += kRedThreads) acc += part[(size_t)c * n + b];
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) out[c] = s;
    }
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
    const dim3 g = gap_grid(nx, ny), b(kRedThreads);
    switch (dual_dtype) {
    case DT_F32:
        hipLaunchKernelGGL((k_gap_part<TV, DT_F32>), g, b, 0, s, nx, ny, B, lam, x, (const float *)p, part);
        break;
    case DT_BF16:
        hipLaunchKernelGGL((k_gap_part<TV, DT_BF16>), g, b, 0, s, nx, ny, B, lam, x, (const uint16_t *)p, part);
        break;
    default:
        hipLaunchKernelGGL((k_gap_part<TV, DT_F16>), g, b, 0, s, nx, ny, B, lam, x, (const _Float16 *)p, part);
        break;
    }
}

} // namespace

int reduce_partial_blocks() { return kRedBlocks; }

size_t gap_partial_doubles(int nx, int ny, int, int)
{
    const dim3 g = gap_grid(nx, ny);
    return 3 * (size_t)g.x * g.y;
}

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
    const dim3 g = gap_grid(nx, ny);
    hipLaunchKernelGGL(k_final_n, dim3(1), dim3(kRedThreads), 0, s, 3, (int)(g.x * g.y), (const double *)partials,
                       out_dev);
    return SCI_OK;
}

} // namespace sci
