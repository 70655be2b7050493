// Fused-schedule TV denoiser kernel (template), instantiated per tile shape
// in the k_fgp_tile_*.hip translation units.
//
// M inner FGP iterations (Algorithm 1, FGP / Cham boxes; projections of
// Eq. (29)-(30)) per pass over HBM. A workgroup owns one 2D tile of one frame
// (ATV and ITV2D treat frames independently): 64*C columns (C adjacent
// columns per lane) by NW*R rows (R consecutive rows per wavefront, NW
// wavefronts stacked vertically). Every pixel's state (x, p, w) lives in
// registers for all M iterations. Neighbours along j come from the thread's
// own registers or, across a lane boundary, from the adjacent lane by a DPP
// wavefront shift; neighbours along i come from the thread's own registers,
// except across wavefront boundaries where one row per wavefront goes
// through LDS. Each iteration spreads the dependency by one pixel, so a tile
// recomputes a halo of M+1 pixels on its top/left side and M on its
// bottom/right side and writes only its interior. Pixels outside the image
// start (and, with the step set to 0 on every dual entry that carries no
// difference, stay) at x = p = 0, which is exactly the zero padding of the
// difference operators.
//
// The per-voxel arithmetic is exactly that of the streaming kernel (same
// helpers, same operand order, no contraction), so with float32 dual storage
// both schedules produce the same bits. WPE is the occupancy hint (waves per
// SIMD) handed to the register allocator.
#pragma once

#include <hip/hip_runtime.h>

#include "sci_internal.h"
#include "sci_math.h"

namespace sci {

// One tile of one frame: (tx, ty) tile coordinates, frame offset fo (in
// elements), V = elements per dual channel of the whole video.
template <int TV, int M, int DT, int R, int NW, int C>
__device__ __forceinline__ void fgp_tile_body(int nx, int ny, int tx, int ty, uint32_t fo, uint32_t V,
                                              const float *__restrict__ x,
                                              const typename Dual<DT>::T *__restrict__ pc,
                                              const typename Dual<DT>::T *__restrict__ pp, int mode,
                                              const TileBeta &bt, float lam, float step,
                                              typename Dual<DT>::T *__restrict__ pn_out,
                                              typename Dual<DT>::T *__restrict__ pp_out,
                                              float *__restrict__ theta_out, float *__restrict__ u_out,
                                              float (*lds_v)[64 * C], float (*lds_t)[64 * C])
{
    using D = Dual<DT>;
    constexpr int TW = 64 * C;              // tile width incl. halo
    constexpr int TXO = TW - 2 * M - 1;     // interior columns per tile
    constexpr int TYO = NW * R - 2 * M - 1; // interior rows per tile
    static_assert(TXO > 0 && TYO > 0, "tile too small for the pass length");

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int j0 = tx * TXO - (M + 1) + lane * C; // column of this lane's first pixel
    const int ibase = ty * TYO - (M + 1) + wv * R;

    bool jin[C], hj[C];
    float step_h[C]; // horizontal differences exist for 0 <= j < ny-1
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        jin[c] = j >= 0 && j < ny;
        hj[c] = j >= 0 && j < ny - 1;
        step_h[c] = hj[c] ? step : 0.0f;
    }

    float xr[R][C], ph[R][C], pv[R][C], wh[R][C], wv_[R][C];
    // Loads first, arithmetic after: every load uses an in-bounds address
    // (the frame's first element stands in for pixels outside the image) and
    // its value is masked afterwards, so that no load waits behind a branch
    // and all of a lane's loads are in flight together.
    uint32_t pixs[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = ibase + r;
        const bool iin = i >= 0 && i < nx;
#pragma unroll
        for (int c = 0; c < C; ++c) pixs[r][c] = (jin[c] && iin) ? (uint32_t)i * ny + (uint32_t)(j0 + c) : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) xr[r][c] = x[fo + pixs[r][c]];
    if (mode == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) ph[r][c] = pv[r][c] = wh[r][c] = wv_[r][c] = 0.0f;
    } else {
        // p^(s0) into ph/pv, p^(s0-1) staged in wh/wv_ (mode 2)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t o = fo + pixs[r][c];
                ph[r][c] = D::ld(pc, o);
                pv[r][c] = D::ld(pc, V + o);
                if (mode == 2) {
                    wh[r][c] = D::ld(pp, o);
                    wv_[r][c] = D::ld(pp, V + o);
                }
            }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = ibase + r;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const bool hin = hj[c] && i >= 0 && i < nx;      // horizontal difference exists
                const bool vin = jin[c] && i >= 0 && i < nx - 1; // vertical difference exists
                ph[r][c] = hin ? ph[r][c] : 0.0f;
                pv[r][c] = vin ? pv[r][c] : 0.0f;
                if (mode == 2) {
                    wh[r][c] = hin ? extrapolate(ph[r][c], wh[r][c], bt.b[0]) : 0.0f;
                    wv_[r][c] = vin ? extrapolate(pv[r][c], wv_[r][c], bt.b[0]) : 0.0f;
                } else {
                    wh[r][c] = ph[r][c];
                    wv_[r][c] = pv[r][c];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = ibase + r;
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (!(jin[c] && i >= 0 && i < nx)) xr[r][c] = 0.0f;
    }

    auto interior = [&](int r, int c) {
        const int cw = lane * C + c, rr = wv * R + r;
        return cw >= M + 1 && cw <= TW - 1 - M && j0 + c < ny && rr >= M + 1 && rr <= NW * R - 1 - M &&
               ibase + r < nx;
    };

#pragma unroll
    for (int t = 0; t < M; ++t) {
        // theta = x - lambda D^T w (w_v of the row above may live in the wavefront above)
#pragma unroll
        for (int c = 0; c < C; ++c) lds_v[wv][lane * C + c] = wv_[R - 1][c];
        __syncthreads();
        float up[C];
#pragma unroll
        for (int c = 0; c < C; ++c) up[c] = wv > 0 ? lds_v[wv - 1][lane * C + c] : 0.0f;
        float th[R][C];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float whl = c > 0 ? wh[r][c - 1] : from_left(wh[r][C - 1]);
                th[r][c] = theta_of(xr[r][c], whl, wh[r][c], r > 0 ? wv_[r - 1][c] : up[c], wv_[r][c], lam);
            }
#pragma unroll
        for (int c = 0; c < C; ++c) lds_t[wv][lane * C + c] = th[0][c];
        __syncthreads();
        float dn[C];
#pragma unroll
        for (int c = 0; c < C; ++c) dn[c] = wv < NW - 1 ? lds_t[wv + 1][lane * C + c] : 0.0f;
        const float bnext = bt.b[t + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = ibase + r;
            const float step_v = (i >= 0 && i < nx - 1) ? step : 0.0f; // uniform per row
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float thr = c < C - 1 ? th[r][c + 1] : from_right(th[r][0]);
                const float zh = thr - th[r][c];
                const float zv = (r < R - 1 ? th[r + 1][c] : dn[c]) - th[r][c];
                const float qh = ascend(wh[r][c], zh, step_h[c]);
                const float qv = ascend(wv_[r][c], zv, step_v);
                float nh, nv;
                if (TV == TV_ATV) {
                    nh = proj_atv(qh);
                    nv = proj_atv(qv);
                } else {
                    const float s = iso_scale(norm2_add(0.0f, qh, qv));
                    nh = qh * s;
                    nv = qv * s;
                }
                if (t == M - 1 && pp_out && interior(r, c)) { // p^(s0+M-1) is about to be replaced
                    const uint32_t o = fo + (uint32_t)i * ny + (j0 + c);
                    D::st(pp_out, o, ph[r][c]);
                    D::st(pp_out, V + o, pv[r][c]);
                }
                wh[r][c] = extrapolate(nh, ph[r][c], bnext);
                wv_[r][c] = extrapolate(nv, pv[r][c], bnext);
                ph[r][c] = nh;
                pv[r][c] = nv;
            }
        }
    }

    if (pn_out) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (interior(r, c)) {
                    const uint32_t o = fo + (uint32_t)(ibase + r) * ny + (j0 + c);
                    D::st(pn_out, o, ph[r][c]);
                    D::st(pn_out, V + o, pv[r][c]);
                }
    }
    if (theta_out) {
        // theta = x - lambda D^T p^(s0+M) with the last projected dual
#pragma unroll
        for (int c = 0; c < C; ++c) lds_v[wv][lane * C + c] = pv[R - 1][c];
        __syncthreads();
        float up[C];
#pragma unroll
        for (int c = 0; c < C; ++c) up[c] = wv > 0 ? lds_v[wv - 1][lane * C + c] : 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float phl = c > 0 ? ph[r][c - 1] : from_left(ph[r][C - 1]);
                const float th = theta_of(xr[r][c], phl, ph[r][c], r > 0 ? pv[r - 1][c] : up[c], pv[r][c], lam);
                if (interior(r, c)) {
                    const uint32_t o = fo + (uint32_t)(ibase + r) * ny + (j0 + c);
                    theta_out[o] = th;
                    if (u_out) u_out[o] = xr[r][c] - th;
                }
            }
    }
}

template <int TV, int M, int DT, int R, int NW, int C, int WPE>
__global__ __launch_bounds__(64 * NW, WPE) void k_fgp_tile(int nx, int ny, int ntx, int ntiles,
                                                           const float *__restrict__ x,
                                                           const typename Dual<DT>::T *__restrict__ pc,
                                                           const typename Dual<DT>::T *__restrict__ pp, int mode,
                                                           TileBeta bt, float lam, float step,
                                                           typename Dual<DT>::T *__restrict__ pn_out,
                                                           typename Dual<DT>::T *__restrict__ pp_out,
                                                           float *__restrict__ theta_out, float *__restrict__ u_out)
{
    __shared__ float lds_v[NW][64 * C]; // last-row vertical dual of each wavefront
    __shared__ float lds_t[NW][64 * C]; // first-row theta of each wavefront
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int frame = lin / ntiles, tile = lin % ntiles;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    fgp_tile_body<TV, M, DT, R, NW, C>(nx, ny, tile % ntx, tile / ntx, (uint32_t)frame * plane,
                                       plane * (gridDim.x / (uint32_t)ntiles), x, pc, pp, mode, bt, lam, step,
                                       pn_out, pp_out, theta_out, u_out, lds_v, lds_t);
}

template <int TV, int M, int DT, int R, int NW, int C, int WPE>
void launch_tile_m(int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    constexpr int TXO = 64 * C - 2 * M - 1, TYO = NW * R - 2 * M - 1;
    const int ntx = (ny + TXO - 1) / TXO, nty = (nx + TYO - 1) / TYO;
    hipLaunchKernelGGL((k_fgp_tile<TV, M, DT, R, NW, C, WPE>), dim3(ntx * nty * B), dim3(64 * NW), 0, s, nx, ny,
                       ntx, ntx * nty, x, (const T *)tp.pc, (const T *)tp.pp, tp.mode, tp.beta, lam,
                       1.0f / (8.0f * lam), (T *)tp.pn_out, (T *)tp.pp_out, tp.theta, tp.u_out);
}

// Dispatch on the pass length m = 1..kTileMaxM for one tile shape.
template <int TV, int DT, int R, int NW, int C, int WPE>
int launch_tile_shape(int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s)
{
    static_assert(kTileMaxM == 10, "pass lengths dispatched below");
    switch (m) {
    case 1: launch_tile_m<TV, 1, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 2: launch_tile_m<TV, 2, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 3: launch_tile_m<TV, 3, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 4: launch_tile_m<TV, 4, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 5: launch_tile_m<TV, 5, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 6: launch_tile_m<TV, 6, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 7: launch_tile_m<TV, 7, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 8: launch_tile_m<TV, 8, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 9: launch_tile_m<TV, 9, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 10: launch_tile_m<TV, 10, DT, R, NW, C, WPE>(nx, ny, B, x, tp, lam, s); return SCI_OK;
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
