// TV denoiser kernels (Algorithm 1 FGP / Cham boxes, dual projections of
// Eq. (29)-(32)), streaming schedule: one pass over HBM per inner iteration.
//
// Mapping. One wavefront owns a strip of 64 consecutive columns and walks
// down a segment of rows. Lane l holds column j = 62*strip - 1 + l, so lanes
// 0 and 63 are halo lanes and lanes 1..62 write results: horizontal
// neighbours come from the adjacent lane by a DPP wavefront shift, vertical
// neighbours from the registers of the previous row. Each row step loads
// p^(s), p^(s-1) (both channels) and x of the NEXT row once, coalesced
// (64 lanes x 4 bytes), rebuilds w and theta for it on chip, and finishes
// the current row: z = D theta, q = w + z/(8 lambda), projection, store.
//
// ATV and ITV2D project each voxel on its own, so a frame is a grid
// dimension and each lane handles one frame. VTV normalises all 2B dual
// values of a pixel together, so each lane carries every frame of its column
// in registers (KB >= B) and projects once all frames of the row are done.
#include <hip/hip_runtime.h>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

constexpr int kWaves = 4;  // wavefronts per workgroup
constexpr int kStrip = 62; // result columns per wavefront

template <int TV, int KB, int DT>
__global__ __launch_bounds__(64 * kWaves) void k_fgp_stream(int nx, int ny, int B, int rows, int nstrips,
                                                            int nwaves, const float *__restrict__ x,
                                                            const typename Dual<DT>::T *__restrict__ pc,
                                                            const typename Dual<DT>::T *__restrict__ pp,
                                                            typename Dual<DT>::T *__restrict__ pn, int mode,
                                                            float beta, float lam, float step)
{
    using D = Dual<DT>;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wave >= nwaves) return; // uniform per wavefront
    const int strip = wave % nstrips;
    const int i0 = (wave / nstrips) * rows;
    const int i1 = min(nx, i0 + rows);
    const int j = strip * kStrip - 1 + lane;
    const bool jin = j >= 0 && j < ny;     // column inside the image
    const bool hin = j >= 0 && j < ny - 1; // column has a horizontal difference
    const bool outl = lane >= 1 && lane <= kStrip && j < ny;
    const float step_h = hin ? step : 0.0f; // no horizontal difference at j = ny-1 (and outside)
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int kbase = (KB == 1) ? (int)blockIdx.y : 0;
    const int nk = (KB == 1) ? 1 : B;

    // w at offset o (channel offset already added), 0 where no difference exists
    auto load_w = [&](uint32_t o, bool valid) -> float {
        if (mode == 0 || !valid) return 0.0f;
        float p = D::ld(pc, o);
        return mode == 2 ? extrapolate(p, D::ld(pp, o), beta) : p;
    };

    float wh0[KB], wv0[KB], th0[KB];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
        if (kk < nk) {
            const uint32_t fo = (uint32_t)(kbase + kk) * plane;
            const float wvm = (i0 >= 1) ? load_w(V + fo + (uint32_t)(i0 - 1) * ny + j, jin) : 0.0f;
            const uint32_t o = fo + (uint32_t)i0 * ny + j;
            wh0[kk] = load_w(o, hin);
            wv0[kk] = load_w(V + o, jin && i0 < nx - 1);
            const float xv = jin ? x[o] : 0.0f;
            th0[kk] = theta_of(xv, from_left(wh0[kk]), wh0[kk], wvm, wv0[kk], lam);
        }
    }

    for (int i = i0; i < i1; ++i) {
        const bool nxt = i + 1 < nx;
        const float step_v = nxt ? step : 0.0f; // no vertical difference in the last row
        float qh[KB], qv[KB];
        float n2 = 0.0f;
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            if (kk < nk) {
                const uint32_t fo = (uint32_t)(kbase + kk) * plane;
                float wh1 = 0.0f, wv1 = 0.0f, th1 = 0.0f;
                if (nxt) {
                    const uint32_t o1 = fo + (uint32_t)(i + 1) * ny + j;
                    wh1 = load_w(o1, hin);
                    wv1 = load_w(V + o1, jin && i + 1 < nx - 1);
                    const float x1 = jin ? x[o1] : 0.0f;
                    th1 = theta_of(x1, from_left(wh1), wh1, wv0[kk], wv1, lam);
                }
                const float zh = from_right(th0[kk]) - th0[kk];
                const float zv = th1 - th0[kk];
                qh[kk] = ascend(wh0[kk], zh, step_h);
                qv[kk] = ascend(wv0[kk], zv, step_v);
                if (TV == TV_VTV) n2 = norm2_add(n2, qh[kk], qv[kk]);
                wh0[kk] = wh1;
                wv0[kk] = wv1;
                th0[kk] = th1;
            }
        }
        const float vsc = (TV == TV_VTV) ? iso_scale(n2) : 1.0f;
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            if (kk < nk) {
                float ph, pv;
                if (TV == TV_ATV) {
                    ph = proj_atv(qh[kk]);
                    pv = proj_atv(qv[kk]);
                } else if (TV == TV_ITV2D) {
                    const float s = iso_scale(norm2_add(0.0f, qh[kk], qv[kk]));
                    ph = qh[kk] * s;
                    pv = qv[kk] * s;
                } else {
                    ph = qh[kk] * vsc;
                    pv = qv[kk] * vsc;
                }
                if (outl) {
                    const uint32_t o = (uint32_t)(kbase + kk) * plane + (uint32_t)i * ny + j;
                    D::st(pn, o, ph);
                    D::st(pn, V + o, pv);
                }
            }
        }
    }
}

// theta = x - lambda D^T p per voxel; optionally u = x - theta.
template <int DT>
__global__ __launch_bounds__(256) void k_tv_theta(int nx, int ny, uint32_t V, const float *__restrict__ x,
                                                  const typename Dual<DT>::T *__restrict__ p, float lam,
                                                  float *__restrict__ theta, float *__restrict__ u_out)
{
    using D = Dual<DT>;
    const uint32_t o = blockIdx.x * 256u + threadIdx.x;
    if (o >= V) return;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t r = o % plane;
    const int i = (int)(r / (uint32_t)ny), j = (int)(r % (uint32_t)ny);
    const float whl = j >= 1 ? D::ld(p, o - 1) : 0.0f;
    const float wh = j < ny - 1 ? D::ld(p, o) : 0.0f;
    const float wvu = i >= 1 ? D::ld(p, V + o - ny) : 0.0f;
    const float wv = i < nx - 1 ? D::ld(p, V + o) : 0.0f;
    const float xv = x[o];
    const float th = theta_of(xv, whl, wh, wvu, wv, lam);
    theta[o] = th;
    if (u_out) u_out[o] = xv - th;
}

int pick_rows(int nx, int nstrips, int frames_in_grid)
{
    // Enough wavefronts to cover the chip several times over; shorter row
    // segments only cost one extra halo row per segment.
    int rows = 64;
    while (rows > 4 && (long)nstrips * frames_in_grid * ((nx + rows - 1) / rows) < 8192) rows >>= 1;
    return rows;
}

template <int TV, int KB, int DT>
void launch_stream_t(int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn, int mode,
                     float beta, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    const int nstrips = (ny + kStrip - 1) / kStrip;
    const int frames = (KB == 1) ? B : 1;
    const int rows = pick_rows(nx, nstrips, frames);
    const int nwaves = nstrips * ((nx + rows - 1) / rows);
    const dim3 grid((nwaves + kWaves - 1) / kWaves, frames);
    hipLaunchKernelGGL((k_fgp_stream<TV, KB, DT>), grid, dim3(64 * kWaves), 0, s, nx, ny, B, rows, nstrips, nwaves,
                       x, (const T *)pc, (const T *)pp, (T *)pn, mode, beta, lam, 1.0f / (8.0f * lam));
}

template <int DT>
int launch_stream_dt(int tv, int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn,
                     int mode, float beta, float lam, hipStream_t s)
{
    if (tv == TV_ATV) {
        launch_stream_t<TV_ATV, 1, DT>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    } else if (tv == TV_ITV2D) {
        launch_stream_t<TV_ITV2D, 1, DT>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    } else if (B <= 8) {
        launch_stream_t<TV_VTV, 8, DT>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    } else if (B <= 16) {
        launch_stream_t<TV_VTV, 16, DT>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    } else if (B <= 32) {
        launch_stream_t<TV_VTV, 32, DT>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    } else {
        return SCI_ERR_UNSUPPORTED;
    }
    return SCI_OK;
}

} // namespace

int launch_fgp_stream(int tv, int dual_dtype, int nx, int ny, int B, const float *x, const void *p_cur,
                      const void *p_prev, void *p_next, int mode, float beta, float lam, hipStream_t s)
{
    switch (dual_dtype) {
    case DT_F32: return launch_stream_dt<DT_F32>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    case DT_BF16: return launch_stream_dt<DT_BF16>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    case DT_F16: return launch_stream_dt<DT_F16>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    }
    return SCI_ERR_INVALID_ARG;
}

int launch_tv_theta(int dual_dtype, int nx, int ny, int B, const float *x, const void *p, float lam, float *theta,
                    float *u_out, hipStream_t s)
{
    const uint32_t V = (uint32_t)nx * (uint32_t)ny * (uint32_t)B;
    const dim3 grid((V + 255u) / 256u);
    switch (dual_dtype) {
    case DT_F32:
        hipLaunchKernelGGL(k_tv_theta<DT_F32>, grid, dim3(256), 0, s, nx, ny, V, x, (const float *)p, lam, theta,
                           u_out);
        return SCI_OK;
    case DT_BF16:
        hipLaunchKernelGGL(k_tv_theta<DT_BF16>, grid, dim3(256), 0, s, nx, ny, V, x, (const uint16_t *)p, lam,
                           theta, u_out);
        return SCI_OK;
    case DT_F16:
        hipLaunchKernelGGL(k_tv_theta<DT_F16>, grid, dim3(256), 0, s, nx, ny, V, x, (const _Float16 *)p, lam,
                           theta, u_out);
        return SCI_OK;
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
