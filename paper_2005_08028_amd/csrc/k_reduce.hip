// FP64 reductions on the GPU: squared differences (PSNR), the measurement
// residual ||Y - Phi X||^2, and the terms of the denoiser's duality gap.
//
// Deterministic two-stage scheme: a fixed grid of workgroups, each thread
// accumulates a fixed slice in double, the workgroup folds its values in a
// fixed order into one partial; a single workgroup then folds the partials
// in the same fixed order. No floating-point atomics, so repeated calls
// return bit-identical results.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// ---- duality-gap terms ----------------------------------------------------
//
// Partials [3][nwg]: TV(theta), <D theta, p>, ||theta - x||^2 with
// theta = x - lambda D^T p, all in FP64. Mapping as in the streaming FGP
// pass: a wavefront owns a strip of 64 columns (62 accumulate, lanes 0 and
// 63 are halo) and walks down a row segment; theta of each voxel is formed
// once, its j+1 neighbour comes from the next lane (DPP), its i+1 neighbour
// from the next row step. The frames of a pixel are split over the
// wavefronts of a workgroup; for VTV their partial sums of |D theta|^2 meet
// in LDS once per row (fixed order) before the square root. Loads come in
// double-buffered 2-row chunks from clamped in-bounds addresses, masked
// where consumed. Every sum runs in a fixed order, so repeated calls return
// bit-identical results.
constexpr int kGapStrip = 62;
constexpr int kGapMaxWaves = 8;
constexpr int kGapChunk = 2;
constexpr int kGapMinRows = 8;

// The value held by lane l+1 (0 in lane 63), for a double.
__device__ inline double from_right_d(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x130, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront by a fixed butterfly; every lane
// ends with the same value.
__device__ inline double wave_sum(double v)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

template <int DT> struct GapRow {
    float x;
    typename Dual<DT>::T ph, pv;
};

template <int TV, int KF, int R, int DT>
__global__ __launch_bounds__(64 * kGapMaxWaves) void k_gap_rows(int nx, int ny, int B, int fpw, int rows,
                                                                 int nstrips, double lam,
                                                                 const float *__restrict__ x,
                                                                 const typename Dual<DT>::T *__restrict__ p,
                                                                 double *__restrict__ part)
{
    using D = Dual<DT>;
    __shared__ double s2s[2][kGapMaxWaves][64];
    __shared__ double red[3][kGapMaxWaves];
    const int ng = (int)(blockDim.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    const int t = xcd_contiguous((int)(blockIdx.x + blockIdx.y * gridDim.x), (int)(gridDim.x * gridDim.y));
    const int fgrp = t / (int)gridDim.x, tile = t % (int)gridDim.x;
    const int strip = tile % nstrips;
    const int i0 = (tile / nstrips) * rows;
    const int i1 = min(nx, i0 + rows);
    const int j = strip * kGapStrip - 1 + lane;
    const bool jin = j >= 0 && j < ny;
    const bool hin = j >= 0 && j < ny - 1; // p_h(i, j) exists; also "j + 1 < ny" for the j-difference
    const bool outl = lane >= 1 && lane <= kGapStrip && j < ny;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int kbase = (fgrp * ng + g) * fpw; // fgrp = 0 for VTV
    // VTV: the sums read all kGapMaxWaves slots in one fixed run; absent
    // wavefronts' slots hold +0 (the first barrier orders these writes)
    if (TV == TV_VTV)
        for (int e = (int)threadIdx.x; e < 2 * kGapMaxWaves * 64; e += (int)blockDim.x)
            if ((e >> 6) % kGapMaxWaves >= ng) (&s2s[0][0][0])[e] = 0.0;
    const int nk = max(0, min(fpw, B - kbase));
    uint32_t fo[KF];
#pragma unroll
    for (int kk = 0; kk < KF; ++kk)
        fo[kk] = (uint32_t)min(kbase + kk, B - 1) * plane + (jin ? (uint32_t)j : 0u);

    auto issue = [&](GapRow<DT> &l, int kk, int i) {
        const uint32_t o = fo[kk] + (uint32_t)i * (uint32_t)ny;
        l.x = x[o];
        l.ph = p[o];
        l.pv = p[V + o];
    };
    // theta of a row from its x, its masked p_h, p_v and the masked p_v of
    // the row above; the terms are added in the order
    // ((p_h(j-1) - p_h(j)) + p_v(i-1)) - p_v(i)
    auto theta = [&](float xv, float ph, float pv_up, float pv) -> double {
        double s = (double)from_left(ph);
        s -= (double)ph;
        s += (double)pv_up;
        s -= (double)pv;
        return (double)xv - lam * s;
    };

    double th0[KF];
    float ph0[KF], pv0[KF], x0[KF];
    {
        GapRow<DT> up[KF], cur[KF];
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            issue(up[kk], kk, max(i0 - 1, 0));
            issue(cur[kk], kk, i0);
        }
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            const float pvu = jin && i0 >= 1 ? D::cvt(up[kk].pv) : 0.0f;
            ph0[kk] = hin ? D::cvt(cur[kk].ph) : 0.0f;
            pv0[kk] = jin && i0 < nx - 1 ? D::cvt(cur[kk].pv) : 0.0f;
            x0[kk] = cur[kk].x;
            th0[kk] = theta(x0[kk], ph0[kk], pvu, pv0[kk]);
        }
    }

    double tv = 0.0, inner = 0.0, fid = 0.0;
    int par = 0;
    const int ilast = min(i1, nx - 1);
    auto issue_chunk = [&](GapRow<DT>(&nb)[R][KF], int ic) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) issue(nb[rr][kk], kk, min(ic + rr + 1, ilast));
    };
    // rows ic .. ic+R-1, using the loaded rows ic+1 .. ic+R
    auto run_chunk = [&](const GapRow<DT>(&nb)[R][KF], int ic) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = ic + rr;
            const bool has_next = i + 1 < nx;
            const bool mh = hin && has_next, mv = jin && i + 1 < nx - 1;
            const bool acc = outl && i < i1;
            double s2 = 0.0;
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                const GapRow<DT> &r1 = nb[rr][kk];
                const float ph1 = mh ? D::cvt(r1.ph) : 0.0f;
                const float pv1 = mv ? D::cvt(r1.pv) : 0.0f;
                const double th1 = theta(r1.x, ph1, pv0[kk], pv1);
                // the lane shift runs on every lane (a disabled source lane
                // would read as 0); the mask selects afterwards
                const double thr = from_right_d(th0[kk]);
                const double gh = hin ? thr - th0[kk] : 0.0;
                const double gv = has_next ? th1 - th0[kk] : 0.0;
                if (acc && kk < nk) {
                    inner += gh * (double)ph0[kk] + gv * (double)pv0[kk];
                    const double dx = th0[kk] - (double)x0[kk];
                    fid += dx * dx;
                    if (TV == TV_ATV) tv += fabs(gh) + fabs(gv);
                    else if (TV == TV_ITV2D) tv += sqrt(gh * gh + gv * gv);
                    else s2 += gh * gh + gv * gv;
                }
                th0[kk] = th1;
                ph0[kk] = ph1;
                pv0[kk] = pv1;
                x0[kk] = r1.x;
            }
            if (TV == TV_VTV) {
                s2s[par][g][lane] = s2;
                lds_barrier();
                if (g == 0 && acc) {
                    double tot = 0.0;
#pragma unroll
                    for (int gg = 0; gg < kGapMaxWaves; ++gg) tot += s2s[par][gg][lane];
                    tv += sqrt(tot);
                }
                par ^= 1;
            }
        }
    };
    GapRow<DT> ba[R][KF], bb[R][KF];
    issue_chunk(ba, i0);
    for (int ic = i0; ic < i1; ic += 2 * R) {
        issue_chunk(bb, ic + R);
        run_chunk(ba, ic);
        issue_chunk(ba, ic + 2 * R);
        run_chunk(bb, ic + R);
    }

    // fixed-order workgroup sums: lanes by butterfly, wavefronts in order
    tv = wave_sum(tv);
    inner = wave_sum(inner);
    fid = wave_sum(fid);
    if (lane == 0) {
        red[0][g] = tv;
        red[1][g] = inner;
        red[2][g] = fid;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b = (int)(blockIdx.x + blockIdx.y * gridDim.x);
        const int nb = (int)(gridDim.x * gridDim.y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double a = 0.0;
            for (int gg = 0; gg < ng; ++gg) a += red[c][gg];
            part[(size_t)c * nb + b] = a;
        }
    }
}

// Launch shape of k_gap_rows: frames per wavefront, wavefronts per
// workgroup, frame groups (grid y), rows per segment, grid x. VTV keeps
// all frames of a pixel in one workgroup (at most 8 x 6 frames); the
// per-voxel TVs take one frame per wavefront.
struct GapShape {
    int fpw, ng, gy, rows, gx, nstrips;
};

GapShape gap_shape(int nx, int ny, int B, int tv)
{
    GapShape sh;
    sh.nstrips = (ny + kGapStrip - 1) / kGapStrip;
    if (tv == TV_VTV) {
        sh.fpw = (B + kGapMaxWaves - 1) / kGapMaxWaves;
        sh.ng = (B + sh.fpw - 1) / sh.fpw;
        sh.gy = 1;
    } else {
        sh.fpw = 1;
        sh.ng = std::min(B, kGapMaxWaves);
        sh.gy = (B + sh.ng - 1) / sh.ng;
    }
    sh.rows = 64;
    while (sh.rows > kGapMinRows && (long)sh.nstrips * sh.gy * ((nx + sh.rows - 1) / sh.rows) < 4096) sh.rows >>= 1;
    sh.gx = sh.nstrips * ((nx + sh.rows - 1) / sh.rows);
    return sh;
}

template <int TV, int KF, int DT>
void launch_gap_rows(const GapShape &sh, int nx, int ny, int B, double lam, const float *x, const void *p,
                     double *part, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    hipLaunchKernelGGL((k_gap_rows<TV, KF, kGapChunk, DT>), dim3(sh.gx, sh.gy), dim3(64 * sh.ng), 0, s, nx, ny, B,
                       sh.fpw, sh.rows, sh.nstrips, lam, x, (const T *)p, part);
}

template <int TV, int DT>
int launch_gap_kf(const GapShape &sh, int nx, int ny, int B, double lam, const float *x, const void *p,
                  double *part, hipStream_t s)
{
    if constexpr (TV != TV_VTV) { // one frame per wavefront
        launch_gap_rows<TV, 1, DT>(sh, nx, ny, B, lam, x, p, part, s);
        return SCI_OK;
    }
    switch (sh.fpw) {
    case 1: launch_gap_rows<TV, 1, DT>(sh, nx, ny, B, lam, x, p, part, s); return SCI_OK;
    case 2: launch_gap_rows<TV, 2, DT>(sh, nx, ny, B, lam, x, p, part, s); return SCI_OK;
    case 3: launch_gap_rows<TV, 3, DT>(sh, nx, ny, B, lam, x, p, part, s); return SCI_OK;
    case 4: launch_gap_rows<TV, 4, DT>(sh, nx, ny, B, lam, x, p, part, s); return SCI_OK;
    case 5:
        if constexpr (TV == TV_VTV) {
            launch_gap_rows<TV, 5, DT>(sh, nx, ny, B, lam, x, p, part, s);
            return SCI_OK;
        }
        break;
    case 6:
        if constexpr (TV == TV_VTV) {
            launch_gap_rows<TV, 6, DT>(sh, nx, ny, B, lam, x, p, part, s);
            return SCI_OK;
        }
        break;
    }
    return SCI_ERR_UNSUPPORTED; // VTV with more than 48 frames
}

template <int TV>
int launch_gap_dt(int dual_dtype, const GapShape &sh, int nx, int ny, int B, double lam, const float *x,
                  const void *p, double *part, hipStream_t s)
{
    switch (dual_dtype) {
    case DT_F32: return launch_gap_kf<TV, DT_F32>(sh, nx, ny, B, lam, x, p, part, s);
    case DT_BF16: return launch_gap_kf<TV, DT_BF16>(sh, nx, ny, B, lam, x, p, part, s);
    case DT_F16: return launch_gap_kf<TV, DT_F16>(sh, nx, ny, B, lam, x, p, part, s);
    }
    return SCI_ERR_INVALID_ARG;
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

} // namespace

int reduce_partial_blocks() { return kRedBlocks; }

size_t gap_partial_doubles(int nx, int ny, int B, int tv)
{
    const GapShape sh = gap_shape(nx, ny, B, tv);
    return 3 * (size_t)sh.gx * sh.gy;
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
    const GapShape sh = gap_shape(nx, ny, B, tv);
    int st;
    if (tv == TV_ATV) st = launch_gap_dt<TV_ATV>(dual_dtype, sh, nx, ny, B, l, x, p, partials, s);
    else if (tv == TV_ITV2D) st = launch_gap_dt<TV_ITV2D>(dual_dtype, sh, nx, ny, B, l, x, p, partials, s);
    else st = launch_gap_dt<TV_VTV>(dual_dtype, sh, nx, ny, B, l, x, p, partials, s);
    if (st != SCI_OK) return st;
    hipLaunchKernelGGL(k_final_n, dim3(1), dim3(kRedThreads), 0, s, 3, sh.gx * sh.gy, (const double *)partials,
                       out_dev);
    return SCI_OK;
}

} // namespace sci
