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
// k_fgp_stream handles one frame per lane (KB = 1) for the per-voxel
// projections; it runs the Chambolle-2004 variant of ATV and ITV2D (their FGP
// passes stream through the 2D tile kernel instead). VTV, which normalises
// all 2B dual values of a pixel together, runs k_vtv_groups: the frames of a
// pixel are split over the wavefronts of a workgroup, which combine their
// partial norms through LDS once per row.
//
// CH = 1 replaces the projection P_K(q) by Chambolle's (2004) semi-implicit
// step p = (w + z/(8 lambda)) / (1 + |z|/(8 lambda)) (Sec. 2.3), with |z|
// taken per component (ATV), per voxel (ITV2D) or per pixel over all frames
// (VTV); it runs on this kernel for every TV kind.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

constexpr int kWaves = 4;  // wavefronts per workgroup
constexpr int kStrip = 62; // result columns per wavefront

// Workgroup barrier over LDS only: waits for this wavefront's LDS accesses
// (lgkmcnt), not for its global loads and stores; the signal fences keep the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F); // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// PF = rows of loads kept in flight ahead of the row being finished (0 for
// VTV, whose B frames per row already give many loads in flight).
//
// Raw loads of one row of one frame: p^(s), p^(s-1) (both channels) and x,
// zero where no difference exists (or outside the image).
struct RowLoad {
    float ph, pv, pph, ppv, x;
};

template <int TV, int KB, int DT, int PF, int CH>
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

    // row i of frame slot kk (i < nx). Loads are issued from in-bounds
    // addresses (the row's first element stands in for columns outside the
    // image) and masked afterwards, so none waits behind a branch.
    auto load_row = [&](int kk, int i) -> RowLoad {
        RowLoad l{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        const uint32_t o = (uint32_t)(kbase + kk) * plane + (uint32_t)i * ny + (jin ? (uint32_t)j : 0u);
        const bool vin = jin && i < nx - 1;
        const float xv = x[o];
        float a = 0.0f, b = 0.0f, c = 0.0f, d = 0.0f;
        if (mode != 0) {
            a = D::ld(pc, o);
            b = D::ld(pc, V + o);
            if (mode == 2) {
                c = D::ld(pp, o);
                d = D::ld(pp, V + o);
            }
        }
        l.x = jin ? xv : 0.0f;
        l.ph = hin ? a : 0.0f;
        l.pv = vin ? b : 0.0f;
        l.pph = hin ? c : 0.0f;
        l.ppv = vin ? d : 0.0f;
        return l;
    };
    auto w_of = [&](float p, float ppv) -> float { return mode == 2 ? extrapolate(p, ppv, beta) : p; };

    float wh0[KB], wv0[KB], th0[KB];
    RowLoad nxt[KB], nxt2[KB];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
        if (kk < nk) {
            float wvm = 0.0f;
            if (i0 >= 1) {
                const RowLoad u = load_row(kk, i0 - 1);
                wvm = w_of(u.pv, u.ppv);
            }
            const RowLoad c = load_row(kk, i0);
            if (PF >= 1 && i0 + 1 < nx) nxt[kk] = load_row(kk, i0 + 1);
            if (PF >= 2 && i0 + 2 < nx) nxt2[kk] = load_row(kk, i0 + 2);
            wh0[kk] = w_of(c.ph, c.pph);
            wv0[kk] = w_of(c.pv, c.ppv);
            th0[kk] = theta_of(c.x, from_left(wh0[kk]), wh0[kk], wvm, wv0[kk], lam);
        }
    }

    for (int i = i0; i < i1; ++i) {
        const bool has_next = i + 1 < nx;
        const float step_v = has_next ? step : 0.0f; // no vertical difference in the last row
        float qh[KB], qv[KB];
        float sh[KB], sv[KB]; // z/(8 lambda) where the difference exists (CH only)
        float n2 = 0.0f;
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            if (kk < nk) {
                // PF = 0: load row i+1 now; PF = 1, 2: it was loaded PF steps ago,
                // and the load PF rows ahead starts here
                RowLoad r1{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (PF == 0) {
                    if (has_next) r1 = load_row(kk, i + 1);
                } else {
                    r1 = nxt[kk];
                    if (PF == 2) {
                        nxt[kk] = nxt2[kk];
                        if (i + 3 < nx && i + 3 <= i1) nxt2[kk] = load_row(kk, i + 3);
                    } else if (i + 2 < nx && i + 2 <= i1) {
                        nxt[kk] = load_row(kk, i + 2);
                    }
                }
                float wh1 = 0.0f, wv1 = 0.0f, th1 = 0.0f;
                if (has_next) {
                    wh1 = w_of(r1.ph, r1.pph);
                    wv1 = w_of(r1.pv, r1.ppv);
                    th1 = theta_of(r1.x, from_left(wh1), wh1, wv0[kk], wv1, lam);
                }
                const float zh = from_right(th0[kk]) - th0[kk];
                const float zv = th1 - th0[kk];
                if (CH) {
                    sh[kk] = step_h * zh;
                    sv[kk] = step_v * zv;
                    qh[kk] = wh0[kk] + sh[kk];
                    qv[kk] = wv0[kk] + sv[kk];
                    if (TV == TV_VTV) n2 = norm2_add(n2, sh[kk], sv[kk]);
                } else {
                    qh[kk] = ascend(wh0[kk], zh, step_h);
                    qv[kk] = ascend(wv0[kk], zv, step_v);
                    if (TV == TV_VTV) n2 = norm2_add(n2, qh[kk], qv[kk]);
                }
                wh0[kk] = wh1;
                wv0[kk] = wv1;
                th0[kk] = th1;
            }
        }
        const float vsc = (TV == TV_VTV) ? (CH ? semi_implicit_scale(n2) : iso_scale(n2)) : 1.0f;
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
            if (kk < nk) {
                float ph, pv;
                if (CH && TV == TV_ATV) {
                    ph = qh[kk] / (1.0f + fabsf(sh[kk]));
                    pv = qv[kk] / (1.0f + fabsf(sv[kk]));
                } else if (CH && TV == TV_ITV2D) {
                    const float s = semi_implicit_scale(norm2_add(0.0f, sh[kk], sv[kk]));
                    ph = qh[kk] * s;
                    pv = qv[kk] * s;
                } else if (TV == TV_ATV) {
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

// VTV with the frames of a pixel split over the NG wavefronts of a
// workgroup: all wavefronts walk the same 62-column strip and row segment,
// wavefront g owning frames [g*fpw, (g+1)*fpw) in registers (KF >= fpw). Per
// row each wavefront forms q for its frames and the partial squared norm
// over them; the partials go through LDS (double-buffered by row parity, one
// barrier per row) and are summed in wavefront order, so every wavefront
// scales its frames by the same per-pixel factor. PF rows of loads are kept
// in flight ahead of the row being finished.
template <int KF, int NG, int DT, int PF, int CH>
__global__ __launch_bounds__(64 * NG) void k_vtv_groups(int nx, int ny, int B, int fpw, int rows, int nstrips,
                                                            const float *__restrict__ x,
                                                            const typename Dual<DT>::T *__restrict__ pc,
                                                            const typename Dual<DT>::T *__restrict__ pp,
                                                            typename Dual<DT>::T *__restrict__ pn, int mode,
                                                            float beta, float lam, float step)
{
    using D = Dual<DT>;
    __shared__ float n2s[2][NG][64];
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    const int strip = (int)blockIdx.x % nstrips;
    const int i0 = ((int)blockIdx.x / nstrips) * rows;
    const int i1 = min(nx, i0 + rows);
    const int j = strip * kStrip - 1 + lane;
    const bool jin = j >= 0 && j < ny;
    const bool hin = j >= 0 && j < ny - 1;
    const bool outl = lane >= 1 && lane <= kStrip && j < ny;
    const float step_h = hin ? step : 0.0f;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int kbase = g * fpw;
    const int nk = max(0, min(fpw, B - kbase)); // frames of this wavefront (0 for a spare one)

    auto load_row = [&](int kk, int i) -> RowLoad {
        RowLoad l{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        const uint32_t o = (uint32_t)(kbase + kk) * plane + (uint32_t)i * ny + j;
        const bool vin = jin && i < nx - 1;
        if (jin) l.x = x[o];
        if (mode != 0) {
            if (hin) l.ph = D::ld(pc, o);
            if (vin) l.pv = D::ld(pc, V + o);
            if (mode == 2) {
                if (hin) l.pph = D::ld(pp, o);
                if (vin) l.ppv = D::ld(pp, V + o);
            }
        }
        return l;
    };
    auto w_of = [&](float p, float ppv) -> float { return mode == 2 ? extrapolate(p, ppv, beta) : p; };

    float wh0[KF], wv0[KF], th0[KF];
    RowLoad nxt[KF];
#pragma unroll
    for (int kk = 0; kk < KF; ++kk) {
        if (kk < nk) {
            float wvm = 0.0f;
            if (i0 >= 1) {
                const RowLoad u = load_row(kk, i0 - 1);
                wvm = w_of(u.pv, u.ppv);
            }
            const RowLoad c = load_row(kk, i0);
            if (PF >= 1 && i0 + 1 < nx) nxt[kk] = load_row(kk, i0 + 1);
            wh0[kk] = w_of(c.ph, c.pph);
            wv0[kk] = w_of(c.pv, c.ppv);
            th0[kk] = theta_of(c.x, from_left(wh0[kk]), wh0[kk], wvm, wv0[kk], lam);
        }
    }

    int par = 0;
    for (int i = i0; i < i1; ++i) {
        const bool has_next = i + 1 < nx;
        const float step_v = has_next ? step : 0.0f;
        float qh[KF], qv[KF];
        float n2 = 0.0f;
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            if (kk < nk) {
                RowLoad r1{0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (PF == 0) {
                    if (has_next) r1 = load_row(kk, i + 1);
                } else {
                    r1 = nxt[kk];
                    if (i + 2 < nx && i + 2 <= i1) nxt[kk] = load_row(kk, i + 2);
                }
                float wh1 = 0.0f, wv1 = 0.0f, th1 = 0.0f;
                if (has_next) {
                    wh1 = w_of(r1.ph, r1.pph);
                    wv1 = w_of(r1.pv, r1.ppv);
                    th1 = theta_of(r1.x, from_left(wh1), wh1, wv0[kk], wv1, lam);
                }
                const float zh = from_right(th0[kk]) - th0[kk];
                const float zv = th1 - th0[kk];
                if (CH) {
                    const float sh = step_h * zh, sv = step_v * zv;
                    qh[kk] = wh0[kk] + sh;
                    qv[kk] = wv0[kk] + sv;
                    n2 = norm2_add(n2, sh, sv);
                } else {
                    qh[kk] = ascend(wh0[kk], zh, step_h);
                    qv[kk] = ascend(wv0[kk], zv, step_v);
                    n2 = norm2_add(n2, qh[kk], qv[kk]);
                }
                wh0[kk] = wh1;
                wv0[kk] = wv1;
                th0[kk] = th1;
            }
        }
        n2s[par][g][lane] = n2;
        lds_barrier();
        float tot = 0.0f;
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) tot += n2s[par][gg][lane];
        const float sc = CH ? semi_implicit_scale(tot) : iso_scale(tot);
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            if (kk < nk && outl) {
                const uint32_t o = (uint32_t)(kbase + kk) * plane + (uint32_t)i * ny + j;
                D::st(pn, o, qh[kk] * sc);
                D::st(pn, V + o, qv[kk] * sc);
            }
        }
        par ^= 1;
    }
}

// theta = x - lambda D^T p per voxel; optionally u = x - theta. Grid:
// column blocks x row strides x frames; loads from in-bounds addresses,
// masked afterwards.
template <int DT>
__global__ __launch_bounds__(256) void k_tv_theta(int nx, int ny, int B, const float *__restrict__ x,
                                                  const typename Dual<DT>::T *__restrict__ p, float lam,
                                                  float *__restrict__ theta, float *__restrict__ u_out)
{
    using D = Dual<DT>;
    const int j = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (j >= ny) return;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const uint32_t fo = (uint32_t)blockIdx.z * plane;
    for (int i = (int)blockIdx.y; i < nx; i += (int)gridDim.y) {
        const uint32_t o = fo + (uint32_t)i * ny + (uint32_t)j;
        const bool l = j >= 1, r = j < ny - 1, u = i >= 1, d = i < nx - 1;
        const float a = D::ld(p, l ? o - 1 : o), b = D::ld(p, o);
        const float c = D::ld(p, V + (u ? o - ny : o)), e = D::ld(p, V + o);
        const float xv = x[o];
        const float th = theta_of(xv, l ? a : 0.0f, r ? b : 0.0f, u ? c : 0.0f, d ? e : 0.0f, lam);
        theta[o] = th;
        if (u_out) u_out[o] = xv - th;
    }
}

int pick_rows(int nx, int nstrips, int frames_in_grid)
{
    // Enough wavefronts to cover the chip several times over; shorter row
    // segments only cost one extra halo row per segment.
    int rows = 64;
    while (rows > 4 && (long)nstrips * frames_in_grid * ((nx + rows - 1) / rows) < 8192) rows >>= 1;
    return rows;
}

template <int TV, int KB, int DT, int CH = 0, int PF = (KB == 1 ? 2 : 0)>
void launch_stream_t(int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn, int mode,
                     float beta, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    const int nstrips = (ny + kStrip - 1) / kStrip;
    const int frames = (KB == 1) ? B : 1;
    const int rows = pick_rows(nx, nstrips, frames);
    const int nwaves = nstrips * ((nx + rows - 1) / rows);
    const dim3 grid((nwaves + kWaves - 1) / kWaves, frames);
    hipLaunchKernelGGL((k_fgp_stream<TV, KB, DT, PF, CH>), grid, dim3(64 * kWaves), 0, s, nx, ny, B, rows, nstrips, nwaves,
                       x, (const T *)pc, (const T *)pp, (T *)pn, mode, beta, lam, 1.0f / (8.0f * lam));
}

constexpr int kVtvWaves = 8; // frame groups (wavefronts) per VTV workgroup

template <int KF, int DT, int CH>
void launch_vtv_t(int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn, int mode,
                  float beta, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    const int nstrips = (ny + kStrip - 1) / kStrip;
    const int fpw = (B + kVtvWaves - 1) / kVtvWaves;
    // enough workgroups to fill the chip several times over
    int rows = 64;
    while (rows > 4 && (long)nstrips * ((nx + rows - 1) / rows) < 2048) rows >>= 1;
    const int nwg = nstrips * ((nx + rows - 1) / rows);
    hipLaunchKernelGGL((k_vtv_groups<KF, kVtvWaves, DT, 1, CH>), dim3(nwg), dim3(64 * kVtvWaves), 0, s, nx, ny, B,
                       fpw, rows,
                       nstrips, x, (const T *)pc, (const T *)pp, (T *)pn, mode, beta, lam, 1.0f / (8.0f * lam));
}

template <int DT, int CH>
int launch_vtv(int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn, int mode, float beta,
               float lam, hipStream_t s)
{
    const int fpw = (B + kVtvWaves - 1) / kVtvWaves;
    if (fpw <= 1) launch_vtv_t<1, DT, CH>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    else if (fpw <= 2) launch_vtv_t<2, DT, CH>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    else if (fpw <= 4) launch_vtv_t<4, DT, CH>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    else return SCI_ERR_UNSUPPORTED;
    return SCI_OK;
}

template <int DT>
int launch_stream_dt(int tv, int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn,
                     int mode, float beta, float lam, hipStream_t s)
{
    // ATV and ITV2D stream through the tile kernel with one iteration per pass
    if (tv == TV_VTV) return launch_vtv<DT, 0>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    return SCI_ERR_UNSUPPORTED;
}

// Chambolle-2004 step, float32 duals, every TV kind
int launch_stream_ch(int tv, int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn,
                     int mode, float beta, float lam, hipStream_t s)
{
    switch (tv) {
    case TV_ATV: launch_stream_t<TV_ATV, 1, DT_F32, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s); return SCI_OK;
    case TV_ITV2D:
        launch_stream_t<TV_ITV2D, 1, DT_F32, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
        return SCI_OK;
    case TV_VTV: return launch_vtv<DT_F32, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace

int launch_fgp_stream_chambolle04(int tv, int dual_dtype, int nx, int ny, int B, const float *x, const void *p_cur,
                                  const void *p_prev, void *p_next, int mode, float beta, float lam, hipStream_t s)
{
    if (dual_dtype != DT_F32) return SCI_ERR_UNSUPPORTED;
    return launch_stream_ch(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
}

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
    const dim3 grid((ny + 255) / 256, (unsigned)std::min(nx, 65535), (unsigned)B);
    switch (dual_dtype) {
    case DT_F32:
        hipLaunchKernelGGL(k_tv_theta<DT_F32>, grid, dim3(256), 0, s, nx, ny, B, x, (const float *)p, lam, theta,
                           u_out);
        return SCI_OK;
    case DT_BF16:
        hipLaunchKernelGGL(k_tv_theta<DT_BF16>, grid, dim3(256), 0, s, nx, ny, B, x, (const uint16_t *)p, lam,
                           theta, u_out);
        return SCI_OK;
    case DT_F16:
        hipLaunchKernelGGL(k_tv_theta<DT_F16>, grid, dim3(256), 0, s, nx, ny, B, x, (const _Float16 *)p, lam,
                           theta, u_out);
        return SCI_OK;
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
