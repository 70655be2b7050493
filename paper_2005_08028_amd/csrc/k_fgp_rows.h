// Row-pipelined fused-schedule TV denoiser kernel (template), instantiated in
// the k_fgp_rows_*.hip translation units; its body also serves the batched
// launch (k_batched.hip).
//
// The same M FGP iterations per pass over HBM as the tiled kernel
// (Algorithm 1, FGP box; projections of Eq. (29)-(30)), decomposed by
// temporal wavefront blocking (Wellein et al., "Efficient temporal blocking
// for stencil computations by multicore-aware wavefront parallelization",
// COMPSAC 2009) instead of overlapped 2D tiles. One wavefront owns a strip of
// 64*C columns of one frame (C adjacent columns per lane; a recomputed halo of
// M+1 columns on the left and M on the right, as in the tiles) and a segment
// of H rows, and walks the segment from top to bottom. Iteration level t
// (0 <= t < M) trails level t-1 by one row: in step k, level t is on row
// r = k - t; it takes w_t and p_t of row r+1, just produced by level t-1 in
// the same step, forms theta_t of row r+1, and with its own theta_t, w_t, p_t
// of row r (kept from the previous step) produces p_{t+1} and w_{t+1} of
// row r for level t+1. All levels of a column live in the lane's registers,
// so rows are recomputed only in the pipeline fill above a segment
// (M+2 rows) and below it (M rows), and no workgroup barrier is needed:
// vertical neighbours are earlier steps of the same lane and horizontal ones
// come from DPP shifts. x of the last rows sits in a ring in LDS private to
// the wavefront, written twice so that every level reads it at a fixed
// offset.
//
// Pixels outside the image hold x = p = 0 and, with the step set to 0 on
// every dual entry that carries no difference, keep p = 0: the zero padding
// of the difference operators. Rows a level computes before the fill has
// reached it hold meaningless values that never enter a stored result (each
// stored value depends only on rows inside its dependency cone). The
// per-voxel arithmetic is that of the streaming and tiled kernels (same
// helpers, same operand order, no contraction), so results are
// bit-identical to theirs with float32 dual storage.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "k_fgp_tile_shapes.h"
#include "sci_internal.h"
#include "sci_math.h"

namespace sci {

constexpr int kRowChunk = 2; // rows loaded per chunk (one chunk ahead)

// f(integral_constant<int, I>) for I = I0 .. N-1, unrolled at compile time.
template <int I0, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I0 < N) {
        f(std::integral_constant<int, I0>{});
        static_for<I0 + 1, N>(f);
    }
}

// LDS ring of rows (x, or starting duals) private to one wavefront.
template <int M, int C> struct alignas(16) RowRing {
    float v[2 * (M + kRowChunk)][64 * C];
};

// The ring padded to 1/8 of a CU's 160 KB of LDS.
template <int M, int C> struct alignas(16) RowRingPadded {
    static constexpr size_t kEighth = 160 * 1024 / 8;
    RowRing<M, C> ring;
    char pad[sizeof(RowRing<M, C>) < kEighth ? kEighth - sizeof(RowRing<M, C>) : 16];
};

// One wavefront's segment: strip sx, segment seg (rows [seg*H, seg*H + H)) of
// the frame at element offset fo; V = elements per dual channel of the whole
// video. MODE: 0 w = 0; 1 w = p^(s0); 2 w = p^(s0) + b[0] (p^(s0) - p^(s0-1)).
// CH_STEP = 1 replaces the projection of q by Chambolle's (2004) semi-implicit step
// p = (w + z/(8 lambda)) / (1 + |z/(8 lambda)|), |.| per component (ATV) or
// per voxel (ITV2D), with the operations of the streaming pass.
// MOM = 0 (no momentum: every beta of the pass is 0, MODE < 2, no p_prev
// output) takes w = p at every level; the extrapolation and the previous
// duals it would read drop out, with identical results.
template <int TV, int M, int DT, int C, int MODE, int CH_STEP = 0, int MOM = 1>
__device__ __forceinline__ void fgp_rows_body(int nx, int ny, int sx, int seg, int H, uint32_t fo, uint32_t V,
                                              const float *__restrict__ x,
                                              const typename Dual<DT>::T *__restrict__ pc,
                                              const typename Dual<DT>::T *__restrict__ pp, const TileBeta &bt,
                                              float lam, float step, typename Dual<DT>::T *__restrict__ pn_out,
                                              typename Dual<DT>::T *__restrict__ pp_out,
                                              float *__restrict__ theta_out, float *__restrict__ u_out,
                                              RowRing<M, C> &rr)
{
    using D = Dual<DT>;
    constexpr int CH = kRowChunk;
    constexpr int TW = 64 * C;
    constexpr int TXO = TW - 2 * M - 1; // interior columns per strip
    constexpr int P = M + CH;           // ring period: rows k+1-M .. k+1 and the chunk written ahead
    static_assert(TXO > 0, "strip too narrow for the pass length");
    auto &ring = rr.v;

    const int lane = threadIdx.x & 63;
    const int a = seg * H;               // first row of the segment
    const int hi = min(a + H, nx);       // one past its last row
    const int j0 = sx * TXO - (M + 1) + lane * C;

    bool jin[C], hj[C], outc[C];
    float step_h[C];
    uint32_t jcl[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        jin[c] = j >= 0 && j < ny;
        hj[c] = j >= 0 && j < ny - 1; // horizontal differences exist for 0 <= j < ny-1
        step_h[c] = hj[c] ? step : 0.0f;
        jcl[c] = jin[c] ? (uint32_t)j : 0u;
        const int cw = lane * C + c;
        outc[c] = cw >= M + 1 && cw <= TW - 1 - M && j < ny;
    }
#pragma unroll
    for (int s = 0; s < 2 * P; ++s)
#pragma unroll
        for (int c = 0; c < C; ++c) ring[s][lane * C + c] = 0.0f;

    // level t's state on its current row r: theta_t(r), w_t(r), p_t(r)
    float cth[M][C], cwh[M][C], cwv[M][C], cph[M][C], cpv[M][C];
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) cth[t][c] = cwh[t][c] = cwv[t][c] = cph[t][c] = cpv[t][c] = 0.0f;
    float cpm[C]; // p_v^(s0+M) of the row above the theta row
#pragma unroll
    for (int c = 0; c < C; ++c) cpm[c] = 0.0f;

    // Chunk loads: x and (MODE >= 1) the starting duals of CH rows, from
    // in-bounds addresses (row 0 / column 0 stand in for pixels outside the
    // image), masked where consumed, so no load sits behind a branch.
    float xn[CH][C], lh[CH][C], lv[CH][C], mh[CH][C], mv[CH][C];
    auto load_chunk = [&](int i0) {
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int i = i0 + s;
            const uint32_t rowo = fo + ((i >= 0 && i < nx) ? (uint32_t)i : 0u) * (uint32_t)ny;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t o = rowo + jcl[c];
                xn[s][c] = x[o];
                if (MODE >= 1) {
                    lh[s][c] = D::ld(pc, o);
                    lv[s][c] = D::ld(pc, V + o);
                }
                if (MODE == 2) {
                    mh[s][c] = D::ld(pp, o);
                    mv[s][c] = D::ld(pp, V + o);
                }
            }
        }
    };

    // Step k runs level t on row k - t. The first stored row a needs level 0
    // from row a - M, primed two steps earlier (theta_0 and w_0 of the row
    // above); the last stored row a+H-1 leaves level M-1 at step a+H+M-2.
    //
    // Relative to k_start, level t first matters at step 2t (it takes in w_t
    // of the row that primes its theta); the first NPRO chunks, where some
    // level is still idle, are unrolled with those levels and the theta
    // stage (whose rows lie above the segment there) left out. Every later
    // chunk runs all levels.
    const int k_start = a - M - 2;
    const int nsteps = H + 2 * M + 1;
    const int nchunk = (nsteps + CH - 1) / CH; // >= M + 1 > NPRO
    constexpr int NPRO = (2 * (M - 1) + CH - 1) / CH;
    load_chunk(k_start + 1);
    auto chunk = [&](int b, auto pro) {
        constexpr int PB = decltype(pro)::value; // prologue chunk index, or -1
        const int k0 = k_start + b * CH;
        // level-0 inputs of the chunk's rows k0+1 .. k0+CH, masked
        float i0h[CH][C], i0v[CH][C], j0h[CH][C], j0v[CH][C];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int i = k0 + s + 1;
            const bool iin = i >= 0 && i < nx;
            const bool ivd = i >= 0 && i < nx - 1;
            const int slot = ((i % P) + P) % P;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float v = (iin && jin[c]) ? xn[s][c] : 0.0f;
                ring[slot][lane * C + c] = v;
                ring[slot + P][lane * C + c] = v;
                const bool hin = iin && hj[c];  // horizontal difference exists
                const bool vin = ivd && jin[c]; // vertical difference exists
                if (MODE == 0) {
                    i0h[s][c] = i0v[s][c] = j0h[s][c] = j0v[s][c] = 0.0f;
                } else {
                    j0h[s][c] = hin ? lh[s][c] : 0.0f;
                    j0v[s][c] = vin ? lv[s][c] : 0.0f;
                    if (MODE == 2) {
                        i0h[s][c] = hin ? extrapolate(j0h[s][c], mh[s][c], bt.b[0]) : 0.0f;
                        i0v[s][c] = vin ? extrapolate(j0v[s][c], mv[s][c], bt.b[0]) : 0.0f;
                    } else {
                        i0h[s][c] = j0h[s][c];
                        i0v[s][c] = j0v[s][c];
                    }
                }
            }
        }
        load_chunk(k0 + CH + 1);
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int k = k0 + s;
            const int base = (((k + 1) % P) + P) % P + P; // x(k+1) in the second copy; x(k+1-t) at base - t
            // inputs of level t: w_t, p_t of row k - t + 1
            float ih[C], iv[C], jh[C], jv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                ih[c] = i0h[s][c];
                iv[c] = i0v[s][c];
                jh[c] = j0h[s][c];
                jv[c] = j0v[s][c];
            }
            float qph[C], qpv[C]; // p^(s0+M-1) of the output row
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (PB >= 0 && PB * CH + s < 2 * t) break; // this level and the later ones are idle
                const int r = k - t;
                // theta_t of row r+1 = x - lambda D^T w_t
                float thn[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float whl = c > 0 ? ih[c - 1] : from_left(ih[C - 1]);
                    thn[c] = theta_of(ring[base - t][lane * C + c], whl, ih[c], cwv[t][c], iv[c], lam);
                }
                const float step_v = (r >= 0 && r < nx - 1) ? step : 0.0f; // uniform per row
                const float bnext = bt.b[t + 1];
                float oh[C], ov[C], nh[C], nv[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float thr = c < C - 1 ? cth[t][c + 1] : from_right(cth[t][0]);
                    const float zh = thr - cth[t][c];
                    const float zv = thn[c] - cth[t][c];
                    if (CH_STEP) {
                        const float sh = step_h[c] * zh, sv = step_v * zv;
                        const float qh = cwh[t][c] + sh, qv = cwv[t][c] + sv;
                        if (TV == TV_ATV) {
                            nh[c] = semi_implicit_atv(qh, sh);
                            nv[c] = semi_implicit_atv(qv, sv);
                        } else {
                            const float s1 = semi_implicit_scale(norm2_add(0.0f, sh, sv));
                            nh[c] = qh * s1;
                            nv[c] = qv * s1;
                        }
                    } else {
                        const float qh = ascend(cwh[t][c], zh, step_h[c]);
                        const float qv = ascend(cwv[t][c], zv, step_v);
                        if (TV == TV_ATV) {
                            nh[c] = proj_atv(qh);
                            nv[c] = proj_atv(qv);
                        } else {
                            const float sc = iso_scale(norm2_add(0.0f, qh, qv));
                            nh[c] = qh * sc;
                            nv[c] = qv * sc;
                        }
                    }
                    if (MOM) {
                        oh[c] = extrapolate(nh[c], cph[t][c], bnext);
                        ov[c] = extrapolate(nv[c], cpv[t][c], bnext);
                    } else {
                        oh[c] = nh[c];
                        ov[c] = nv[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (t == M - 1) {
                        qph[c] = cph[t][c];
                        qpv[c] = cpv[t][c];
                    }
                    cth[t][c] = thn[c];
                    cwh[t][c] = ih[c];
                    cwv[t][c] = iv[c];
                    cph[t][c] = jh[c];
                    cpv[t][c] = jv[c];
                    ih[c] = oh[c];
                    iv[c] = ov[c];
                    jh[c] = nh[c];
                    jv[c] = nv[c];
                }
            }
            if (PB >= 0) continue; // the theta row is above the segment
            // row r = k - M + 1 now has p^(s0+M) in jh, jv: theta = x - lambda D^T p
            const int r = k - M + 1;
            float th[C], xr[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float phl = c > 0 ? jh[c - 1] : from_left(jh[C - 1]);
                xr[c] = ring[base - M][lane * C + c];
                th[c] = theta_of(xr[c], phl, jh[c], cpm[c], jv[c], lam);
                cpm[c] = jv[c];
            }
            if (r >= a && r < hi) { // uniform
                const uint32_t rowo = fo + (uint32_t)r * (uint32_t)ny;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (!outc[c]) continue;
                    const uint32_t o = rowo + (uint32_t)(j0 + c);
                    if (theta_out) theta_out[o] = th[c];
                    if (u_out) u_out[o] = xr[c] - th[c];
                    if (pn_out) {
                        D::st(pn_out, o, jh[c]);
                        D::st(pn_out, V + o, jv[c]);
                    }
                    if (MOM && pp_out) {
                        D::st(pp_out, o, qph[c]);
                        D::st(pp_out, V + o, qpv[c]);
                    }
                }
            }
        }
    };
    static_for<0, NPRO>([&](auto pb) { chunk(decltype(pb)::value, pb); });
    for (int b = NPRO; b < nchunk; ++b) chunk(b, std::integral_constant<int, -1>{});
}

// One pass over every frame: a one-wavefront workgroup per (frame, segment,
// strip), numbered XCD-contiguously.
template <int TV, int M, int DT, int C, int MODE, int CH_STEP, int MOM>
__global__ __launch_bounds__(64, 2) void k_fgp_rows(int nx, int ny, int nstrip, int nseg, int H,
                                                    const float *__restrict__ x,
                                                    const typename Dual<DT>::T *__restrict__ pc,
                                                    const typename Dual<DT>::T *__restrict__ pp, TileBeta bt,
                                                    float lam, float step, typename Dual<DT>::T *__restrict__ pn_out,
                                                    typename Dual<DT>::T *__restrict__ pp_out,
                                                    float *__restrict__ theta_out, float *__restrict__ u_out)
{
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int per_frame = nstrip * nseg;
    const int frame = lin / per_frame, rem = lin % per_frame;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    auto body = [&](RowRing<M, C> &ring) {
        fgp_rows_body<TV, M, DT, C, MODE, CH_STEP, MOM>(nx, ny, rem % nstrip, rem / nstrip, H,
                                                        (uint32_t)frame * plane,
                                                        plane * (gridDim.x / (uint32_t)per_frame), x, pc, pp, bt, lam,
                                                        step, pn_out, pp_out, theta_out, u_out, ring);
    };
    if constexpr (MOM) {
        __shared__ RowRing<M, C> ring;
        body(ring);
    } else {
        // The momentum-free kernel needs few enough registers for three
        // wavefronts per SIMD; its one-wavefront workgroups then spread
        // unevenly over the SIMDs (some run three: 309 against 238 us for a
        // 10-iteration ITV2D pass at 1024x1024x24 inside GAP), so its LDS is
        // padded to admit at most eight workgroups (two wavefronts per SIMD)
        // per CU. The asm keeps the unused padding allocated.
        __shared__ RowRingPadded<M, C> lds;
        asm volatile("; lds padding %0" ::"v"((uint32_t)(size_t)&lds.pad[0]));
        body(lds.ring);
    }
}

// Launch of one pass over every frame: strips of 64*C - 2M - 1 interior
// columns, segments of H rows. The Chambolle-2004 step without momentum
// runs the MOM = 0 instantiation.
template <int TV, int M, int DT, int C, int CH_STEP>
void launch_rows_m(int H, int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s)
{
    using T = typename Dual<DT>::T;
    constexpr int TXO = 64 * C - 2 * M - 1;
    const int nstrip = (ny + TXO - 1) / TXO, nseg = (nx + H - 1) / H;
    const dim3 g(nstrip * nseg * B), b(64);
    const float step = 1.0f / (8.0f * lam);
    bool mom = tp.mode == 2 || tp.pp_out != nullptr;
    for (int t = 1; t <= M; ++t) mom = mom || tp.beta.b[t] != 0.0f;
#define SCI_ROWS_MODE(md, mo)                                                                                       \
    hipLaunchKernelGGL((k_fgp_rows<TV, M, DT, C, md, CH_STEP, mo>), g, b, 0, s, nx, ny, nstrip, nseg, H, x,          \
                       (const T *)tp.pc, (const T *)tp.pp, tp.beta, lam, step, (T *)tp.pn_out, (T *)tp.pp_out,      \
                       tp.theta, tp.u_out)
    if (CH_STEP && !mom) {
        if (tp.mode == 0) SCI_ROWS_MODE(0, 0);
        else SCI_ROWS_MODE(1, 0);
    } else if (tp.mode == 0) SCI_ROWS_MODE(0, 1);
    else if (tp.mode == 1) SCI_ROWS_MODE(1, 1);
    else SCI_ROWS_MODE(2, 1);
#undef SCI_ROWS_MODE
}

// Dispatch on the pass length m = 1..kTileMaxM.
template <int TV, int DT, int CH_STEP = 0>
int launch_rows(int H, int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s)
{
    static_assert(kTileMaxM == 10, "pass lengths dispatched below");
    constexpr int C = kRowCols;
    switch (m) {
    case 1: launch_rows_m<TV, 1, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 2: launch_rows_m<TV, 2, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 3: launch_rows_m<TV, 3, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 4: launch_rows_m<TV, 4, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 5: launch_rows_m<TV, 5, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 6: launch_rows_m<TV, 6, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 7: launch_rows_m<TV, 7, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 8: launch_rows_m<TV, 8, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 9: launch_rows_m<TV, 9, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    case 10: launch_rows_m<TV, 10, DT, C, CH_STEP>(H, nx, ny, B, x, tp, lam, s); return SCI_OK;
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
