// TV denoiser kernels (Algorithm 1 FGP / Cham boxes, dual projections of
// Eq. (29)-(32)), streaming schedule: one pass over HBM per inner iteration.
//
// Mapping. One wavefront owns a strip of 64 consecutive columns and walks
// down a segment of rows. Lane l holds column j = 62*strip - 1 + l, so lanes
// 0 and 63 are halo lanes and lanes 1..62 write results: horizontal
// neighbours come from the adjacent lane by a DPP wavefront shift, vertical
// neighbours from the registers of the previous row. Every value of p^(s),
// p^(s-1) (both channels) and x is loaded once per pass, coalesced (64 lanes
// x 4 bytes), plus one halo row per row segment; each row step rebuilds w
// and theta of the next row on chip and finishes the current row:
// z = D theta, q = w + z/(8 lambda), projection, store.
//
// k_fgp_groups splits the frames of a pixel over the wavefronts of a
// workgroup. VTV, which normalises all 2B dual values of a pixel together,
// combines the wavefronts' partial norms through LDS once per row; the
// library also runs the Chambolle-2004 variant of ATV and ITV2D on it (their
// FGP passes stream through the 2D tile kernel instead).
//
// CH = 1 replaces the projection P_K(q) by Chambolle's (2004) semi-implicit
// step p = (w + z/(8 lambda)) / (1 + |z|/(8 lambda)) (Sec. 2.3), with |z|
// taken per component (ATV), per voxel (ITV2D) or per pixel over all frames
// (VTV).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

constexpr int kStrip = 62; // result columns per wavefront
constexpr int kMaxWaves = 8;  // frame groups (wavefronts) per workgroup, at most

// Streaming pass with the frames of a pixel split over the wavefronts of a
// workgroup (ng = blockDim.x / 64 of them, at most kMaxWaves): all
// wavefronts walk the same 62-column strip and row segment, wavefront g
// owning frames [k0, k0 + fpw), k0 = (fgrp*ng + g)*fpw, in registers
// (KF >= fpw slots; a slot past the last frame reads frame B-1 and neither
// stores nor enters the norm). VTV keeps all frames of a pixel in one
// workgroup (fgrp = 0): per row each wavefront forms q for its frames and
// the partial squared norm over them; the partials of a chunk's R rows go
// through LDS together (double-buffered by chunk parity, one barrier per
// chunk) and are summed in wavefront order, so every wavefront scales its
// frames by the same per-pixel factor. The per-voxel TVs (ATV, ITV2D) take one frame per
// wavefront, frame groups along blockIdx.y, and need no exchange and no
// barrier.
//
// Loads come in chunks of R rows, double-buffered: the raw values of the
// next chunk are issued together, unconditionally, from in-bounds addresses
// (rows past the segment repeat its last needed row, columns outside the
// image read column 0) before the current chunk is finished, so a
// wavefront keeps up to 2R rows of loads in flight. Dual
// values are masked where they are consumed. x is not masked: theta at a
// column or row outside the image enters only differences that are
// multiplied by a zero step (finite input assumed, as everywhere). MODE is
// the pass kind (0: w = 0, 1: w = p, 2: w extrapolated), fixed per launch so
// that no load sits behind a branch.
template <int DT> struct RawRow {
    float x;
    typename Dual<DT>::T ph, pv, pph, ppv;
};

template <int TV, int KF, int R, int DT, int CH, int MODE>
__global__ __launch_bounds__(64 * kMaxWaves) void k_fgp_groups(int nx, int ny, int B, int fpw, int rows,
                                                                  int nstrips, const float *__restrict__ x,
                                                                  const typename Dual<DT>::T *__restrict__ pc,
                                                                  const typename Dual<DT>::T *__restrict__ pp,
                                                                  typename Dual<DT>::T *__restrict__ pn, float beta,
                                                                  float lam, float step)
{
    using D = Dual<DT>;
    __shared__ float n2s[2][kMaxWaves][R][64];
    const int ng = (int)(blockDim.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    // XCD-contiguous numbering over (frame group, segment, strip): adjacent
    // strips, whose loads share the 128-byte lines at their edges, run on
    // one XCD
    const int t = xcd_contiguous((int)(blockIdx.x + blockIdx.y * gridDim.x), (int)(gridDim.x * gridDim.y));
    const int fgrp = t / (int)gridDim.x, tile = t % (int)gridDim.x;
    const int strip = tile % nstrips;
    const int i0 = (tile / nstrips) * rows;
    const int kbase = (fgrp * ng + g) * fpw; // fgrp = 0 for VTV
    const int i1 = min(nx, i0 + rows);
    const int j = strip * kStrip - 1 + lane;
    const bool jin = j >= 0 && j < ny;
    const bool hin = j >= 0 && j < ny - 1;
    const bool outl = lane >= 1 && lane <= kStrip && j < ny;
    const float step_h = hin ? step : 0.0f;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int nk = max(0, min(fpw, B - kbase)); // real frames of this wavefront
    // VTV: every exchange reads all kMaxWaves slots in one fixed run (no loop
    // over ng); absent wavefronts' slots hold +0, which leaves the
    // non-negative sum unchanged. The first exchange's barrier orders these
    // writes before any read.
    if (TV == TV_VTV)
        for (int e = (int)threadIdx.x; e < 2 * kMaxWaves * R * 64; e += (int)blockDim.x)
            if ((e / (R * 64)) % kMaxWaves >= ng) (&n2s[0][0][0][0])[e] = 0.0f;
    uint32_t fo[KF];
#pragma unroll
    for (int kk = 0; kk < KF; ++kk)
        fo[kk] = (uint32_t)min(kbase + kk, B - 1) * plane + (jin ? (uint32_t)j : 0u);

    // raw values of row i (0 <= i < nx) of slot kk
    auto issue = [&](RawRow<DT> &l, int kk, int i) {
        const uint32_t o = fo[kk] + (uint32_t)i * (uint32_t)ny;
        l.x = x[o];
        if (MODE >= 1) {
            l.ph = pc[o];
            l.pv = pc[V + o];
        }
        if (MODE == 2) {
            l.pph = pp[o];
            l.ppv = pp[V + o];
        }
    };
    // w of a loaded row, zero where mask m says the difference does not
    // exist (every value is formed; the masks select, so no load is only
    // used under a branch)
    auto wh_of = [&](const RawRow<DT> &l, bool m) -> float {
        if (MODE == 0) return 0.0f;
        const float p = m ? D::cvt(l.ph) : 0.0f;
        if (MODE == 1) return p;
        return extrapolate(p, m ? D::cvt(l.pph) : 0.0f, beta);
    };
    auto wv_of = [&](const RawRow<DT> &l, bool m) -> float {
        if (MODE == 0) return 0.0f;
        const float p = m ? D::cvt(l.pv) : 0.0f;
        if (MODE == 1) return p;
        return extrapolate(p, m ? D::cvt(l.ppv) : 0.0f, beta);
    };

    float wh0[KF], wv0[KF], th0[KF];
    {
        RawRow<DT> up[KF], cur[KF];
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            issue(up[kk], kk, max(i0 - 1, 0));
            issue(cur[kk], kk, i0);
        }
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            const float wvm = wv_of(up[kk], jin && i0 >= 1);
            wh0[kk] = wh_of(cur[kk], hin);
            wv0[kk] = wv_of(cur[kk], jin && i0 < nx - 1);
            th0[kk] = theta_of(cur[kk].x, from_left(wh0[kk]), wh0[kk], wvm, wv0[kk], lam);
        }
    }

    // rows past the segment's end (and the image's) repeat its last needed
    // row: loaded, never stored
    const int ilast = min(i1, nx - 1);
    auto issue_chunk = [&](RawRow<DT>(&nb)[R][KF], int ic) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) issue(nb[rr][kk], kk, min(ic + rr + 1, ilast));
    };
    int par = 0;
    // finish rows ic .. ic+R-1 from the loaded rows ic+1 .. ic+R: q of all R
    // rows first (row i+1's theta uses the old w only), then, for VTV, one
    // exchange of the R rows' partial norms behind one barrier, then the
    // projections and stores
    auto run_chunk = [&](const RawRow<DT>(&nb)[R][KF], int ic) {
        float qh[R][KF], qv[R][KF];
        float sh[R][KF], sv[R][KF]; // z/(8 lambda) where the difference exists (CH only)
        float n2[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = ic + rr;
            const bool has_next = i + 1 < nx;
            const float step_v = has_next ? step : 0.0f;
            // masks of row i+1 (past the last row every w is 0 there and z_v
            // of row i is multiplied by step_v = 0)
            const bool mh = hin && has_next, mv = jin && i + 1 < nx - 1;
            n2[rr] = 0.0f;
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                const RawRow<DT> &r1 = nb[rr][kk];
                const float wh1 = wh_of(r1, mh);
                const float wv1 = wv_of(r1, mv);
                const float th1 = theta_of(r1.x, from_left(wh1), wh1, wv0[kk], wv1, lam);
                const float zh = from_right(th0[kk]) - th0[kk];
                const float zv = th1 - th0[kk];
                if (CH) {
                    sh[rr][kk] = step_h * zh;
                    sv[rr][kk] = step_v * zv;
                    qh[rr][kk] = wh0[kk] + sh[rr][kk];
                    qv[rr][kk] = wv0[kk] + sv[rr][kk];
                    if (TV == TV_VTV && kk < nk) n2[rr] = norm2_add(n2[rr], sh[rr][kk], sv[rr][kk]);
                } else {
                    qh[rr][kk] = ascend(wh0[kk], zh, step_h);
                    qv[rr][kk] = ascend(wv0[kk], zv, step_v);
                    if (TV == TV_VTV && kk < nk) n2[rr] = norm2_add(n2[rr], qh[rr][kk], qv[rr][kk]);
                }
                wh0[kk] = wh1;
                wv0[kk] = wv1;
                th0[kk] = th1;
            }
        }
        float sc[R];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) sc[rr] = 1.0f;
        if (TV == TV_VTV) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) n2s[par][g][rr][lane] = n2[rr];
            lds_barrier();
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                float tot = 0.0f;
#pragma unroll
                for (int gg = 0; gg < kMaxWaves; ++gg) tot += n2s[par][gg][rr][lane];
                sc[rr] = CH ? semi_implicit_scale(tot) : iso_scale(tot);
            }
            par ^= 1;
        }
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const int i = ic + rr;
            if (i < i1 && outl) {
#pragma unroll
                for (int kk = 0; kk < KF; ++kk) {
                    if (kk < nk) {
                        float ph, pv;
                        if (TV == TV_VTV) {
                            ph = qh[rr][kk] * sc[rr];
                            pv = qv[rr][kk] * sc[rr];
                        } else if (CH && TV == TV_ATV) {
                            ph = semi_implicit_atv(qh[rr][kk], sh[rr][kk]);
                            pv = semi_implicit_atv(qv[rr][kk], sv[rr][kk]);
                        } else if (CH) {
                            const float s1 = semi_implicit_scale(norm2_add(0.0f, sh[rr][kk], sv[rr][kk]));
                            ph = qh[rr][kk] * s1;
                            pv = qv[rr][kk] * s1;
                        } else if (TV == TV_ATV) {
                            ph = proj_atv(qh[rr][kk]);
                            pv = proj_atv(qv[rr][kk]);
                        } else {
                            const float s1 = iso_scale(norm2_add(0.0f, qh[rr][kk], qv[rr][kk]));
                            ph = qh[rr][kk] * s1;
                            pv = qv[rr][kk] * s1;
                        }
                        const uint32_t o = fo[kk] + (uint32_t)i * (uint32_t)ny;
                        D::st(pn, o, ph);
                        D::st(pn, V + o, pv);
                    }
                }
            }
        }
    };
    // two chunk buffers: the loads of one chunk are in flight while the
    // other is finished
    RawRow<DT> ba[R][KF], bb[R][KF];
    issue_chunk(ba, i0);
    for (int ic = i0; ic < i1; ic += 2 * R) {
        issue_chunk(bb, ic + R);
        run_chunk(ba, ic);
        issue_chunk(ba, ic + 2 * R);
        run_chunk(bb, ic + R);
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

constexpr int kChunkRows = 2; // rows per load chunk of k_fgp_groups
constexpr int kMinRows = 8;   // shortest row segment (a multiple of 2 chunks)

template <int TV, int KF, int DT, int CH, int MODE>
void launch_groups_t(int nx, int ny, int B, int fpw, int ng, int gy, const float *x, const void *pc, const void *pp,
                     void *pn, float beta, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    const int nstrips = (ny + kStrip - 1) / kStrip;
    // enough workgroups to fill the chip several times over; segments are
    // whole pairs of chunks
    int rows = 64;
    while (rows > kMinRows && (long)nstrips * gy * ((nx + rows - 1) / rows) < 4096) rows >>= 1;
    const dim3 grid((unsigned)(nstrips * ((nx + rows - 1) / rows)), (unsigned)gy);
    hipLaunchKernelGGL((k_fgp_groups<TV, KF, kChunkRows, DT, CH, MODE>), grid, dim3(64 * ng), 0, s, nx, ny, B, fpw,
                       rows, nstrips, x, (const T *)pc, (const T *)pp, (T *)pn, beta, lam, 1.0f / (8.0f * lam));
}

template <int TV, int KF, int DT, int CH>
void launch_groups_mode(int nx, int ny, int B, int fpw, int ng, int gy, const float *x, const void *pc,
                        const void *pp, void *pn, int mode, float beta, float lam, hipStream_t s)
{
    if (mode == 0) launch_groups_t<TV, KF, DT, CH, 0>(nx, ny, B, fpw, ng, gy, x, pc, pp, pn, beta, lam, s);
    else if (mode == 1) launch_groups_t<TV, KF, DT, CH, 1>(nx, ny, B, fpw, ng, gy, x, pc, pp, pn, beta, lam, s);
    else launch_groups_t<TV, KF, DT, CH, 2>(nx, ny, B, fpw, ng, gy, x, pc, pp, pn, beta, lam, s);
}

// VTV: B split over at most kMaxWaves wavefronts of one workgroup (at most
// 6 frames each). Per-voxel TVs: one frame per wavefront, kMaxWaves
// wavefronts per workgroup, frame groups along blockIdx.y.
template <int TV, int DT, int CH>
int launch_groups(int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn, int mode,
                  float beta, float lam, hipStream_t s)
{
    if (TV != TV_VTV) {
        const int ng = std::min(B, kMaxWaves);
        launch_groups_mode<TV, 1, DT, CH>(nx, ny, B, 1, ng, (B + ng - 1) / ng, x, pc, pp, pn, mode, beta, lam, s);
        return SCI_OK;
    }
    const int fpw = (B + kMaxWaves - 1) / kMaxWaves;
    const int ng = (B + fpw - 1) / fpw;
    switch (fpw) {
    case 1: launch_groups_mode<TV, 1, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s); return SCI_OK;
    case 2: launch_groups_mode<TV, 2, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s); return SCI_OK;
    case 3: launch_groups_mode<TV, 3, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s); return SCI_OK;
    case 4: launch_groups_mode<TV, 4, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s); return SCI_OK;
    case 5:
        if constexpr (TV == TV_VTV) {
            launch_groups_mode<TV, 5, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s);
            return SCI_OK;
        }
        break;
    case 6:
        if constexpr (TV == TV_VTV) {
            launch_groups_mode<TV, 6, DT, CH>(nx, ny, B, fpw, ng, 1, x, pc, pp, pn, mode, beta, lam, s);
            return SCI_OK;
        }
        break;
    }
    return SCI_ERR_UNSUPPORTED; // more than 48 frames
}

template <int DT>
int launch_stream_dt(int tv, int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn,
                     int mode, float beta, float lam, hipStream_t s)
{
    // ATV and ITV2D stream through the tile kernel with one iteration per pass
    if (tv == TV_VTV) return launch_groups<TV_VTV, DT, 0>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    return SCI_ERR_UNSUPPORTED;
}

// Chambolle-2004 step, every TV kind and storage type
template <int DT>
int launch_stream_ch(int tv, int nx, int ny, int B, const float *x, const void *pc, const void *pp, void *pn,
                     int mode, float beta, float lam, hipStream_t s)
{
    switch (tv) {
    case TV_ATV: return launch_groups<TV_ATV, DT, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    case TV_ITV2D: return launch_groups<TV_ITV2D, DT, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    case TV_VTV: return launch_groups<TV_VTV, DT, 1>(nx, ny, B, x, pc, pp, pn, mode, beta, lam, s);
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace

int launch_fgp_stream_chambolle04(int tv, int dual_dtype, int nx, int ny, int B, const float *x, const void *p_cur,
                                  const void *p_prev, void *p_next, int mode, float beta, float lam, hipStream_t s)
{
    switch (dual_dtype) {
    case DT_F32: return launch_stream_ch<DT_F32>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    case DT_BF16: return launch_stream_ch<DT_BF16>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    case DT_F16: return launch_stream_ch<DT_F16>(tv, nx, ny, B, x, p_cur, p_prev, p_next, mode, beta, lam, s);
    }
    return SCI_ERR_UNSUPPORTED;
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
