// Row-pipelined ATV-Clip passes (Sec. 2.3; Algorithm 1, Clip box): M clipping
// iterations per pass over HBM, float32 duals.
//
// The two difference directions never interact, which shapes the kernel:
//   * vertical duals couple only along a column, so they are pipelined down
//     a row segment like the FGP row kernel (k_fgp_rows.h): level t is one row
//     behind level t-1 and keeps w_v of its current row and the row above;
//   * horizontal duals couple only along a row, so when a row leaves the
//     vertical pipeline its M horizontal iterations run at once in registers,
//     neighbours by DPP across lanes.
// A wavefront owns a strip of 64*C columns (a recomputed halo of M+1 columns
// on the left and M on the right) and a segment of H rows of one frame; x
// rows (and, for a warm start, the starting horizontal duals) sit in LDS
// rings private to the wavefront. Each update is the streaming kernel's
// expression (k_clip.hip) and theta that of the theta pass, so the results are
// bit-identical to one pass per iteration.
#include <hip/hip_runtime.h>

#include "k_fgp_rows.h"
#include "sci_internal.h"
#include "sci_math.h"

namespace sci {
namespace {

__device__ inline float clip_to(float v, float T) { return fminf(fmaxf(v, -T), T); }

// MODE: 0 every dual starts at 0; 1 from w_in (two channels, h then v).
template <int M, int C, int MODE>
__global__ __launch_bounds__(64, 2) void k_clip_rows(int nx, int ny, int nstrip, int nseg, int H,
                                                     const float *__restrict__ x, const float *__restrict__ w_in,
                                                     float inv_alpha, float T, float *__restrict__ w_out,
                                                     float *__restrict__ theta_out, float *__restrict__ u_out)
{
    constexpr int CH = kRowChunk;
    constexpr int TW = 64 * C;
    constexpr int TXO = TW - 2 * M - 1; // interior columns per strip
    constexpr int P = M + CH;           // ring period: rows k+1-M .. k+1 and the chunk written ahead
    static_assert(TXO > 0, "strip too narrow for the pass length");
    __shared__ RowRing<M, C> xring;
    __shared__ RowRing<(MODE == 1 ? M : 0), C> hring; // starting horizontal duals (warm start)
    auto &ring = xring.v;

    const int lane = threadIdx.x & 63;
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int per_frame = nstrip * nseg;
    const int frame = lin / per_frame, rem = lin % per_frame;
    const int seg = rem / nstrip, sx = rem % nstrip;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t fo = (uint32_t)frame * plane;
    const uint32_t V = plane * (gridDim.x / (uint32_t)per_frame);
    const int a = seg * H;         // first row of the segment
    const int hi = min(a + H, nx); // one past its last row
    const int j0 = sx * TXO - (M + 1) + lane * C;

    bool jin[C], hd[C], outc[C];
    uint32_t jcl[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = j0 + c;
        jin[c] = j >= 0 && j < ny;
        hd[c] = j >= 0 && j < ny - 1; // a horizontal difference exists
        jcl[c] = jin[c] ? (uint32_t)j : 0u;
        const int cw = lane * C + c;
        outc[c] = cw >= M + 1 && cw <= TW - 1 - M && j < ny;
    }
#pragma unroll
    for (int s = 0; s < 2 * P; ++s)
#pragma unroll
        for (int c = 0; c < C; ++c) {
            ring[s][lane * C + c] = 0.0f;
            if constexpr (MODE == 1) hring.v[s][lane * C + c] = 0.0f;
        }

    // vertical level t on its row r: w_v of rows r-1 and r
    float wvm[M][C], wv0[M][C];
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int c = 0; c < C; ++c) wvm[t][c] = wv0[t][c] = 0.0f;
    float cpm[C]; // final w_v of the row above the theta row
#pragma unroll
    for (int c = 0; c < C; ++c) cpm[c] = 0.0f;

    float xn[CH][C], lh[CH][C], lv[CH][C];
    auto load_chunk = [&](int i0) {
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int i = i0 + s;
            const uint32_t rowo = fo + ((i >= 0 && i < nx) ? (uint32_t)i : 0u) * (uint32_t)ny;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t o = rowo + jcl[c];
                xn[s][c] = x[o];
                if constexpr (MODE == 1) {
                    lh[s][c] = w_in[o];
                    lv[s][c] = w_in[V + o];
                }
            }
        }
    };

    const int k_start = a - M - 2;
    const int nsteps = H + 2 * M + 1;
    const int nchunk = (nsteps + CH - 1) / CH; // >= M + 1 > NPRO
    constexpr int NPRO = (2 * (M - 1) + CH - 1) / CH;
    load_chunk(k_start + 1);
    auto chunk = [&](int b, auto pro) {
        constexpr int PB = decltype(pro)::value; // prologue chunk index, or -1
        const int k0 = k_start + b * CH;
        float v0in[CH][C]; // starting w_v of the chunk's rows (level-0 input)
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
                if constexpr (MODE == 1) {
                    const float h = (iin && hd[c]) ? lh[s][c] : 0.0f;
                    hring.v[slot][lane * C + c] = h;
                    hring.v[slot + P][lane * C + c] = h;
                    v0in[s][c] = (ivd && jin[c]) ? lv[s][c] : 0.0f;
                } else {
                    v0in[s][c] = 0.0f;
                }
            }
        }
        load_chunk(k0 + CH + 1);
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int k = k0 + s;
            const int base = (((k + 1) % P) + P) % P + P; // x(k+1) in the second copy; x(k+1-t) at base - t
            float in[C];                                  // w_v of row r+1 for level t
#pragma unroll
            for (int c = 0; c < C; ++c) in[c] = v0in[s][c];
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (PB >= 0 && PB * CH + s < 2 * t) break; // this level and the later ones are idle
                const int r = k - t;
                const bool vd = r >= 0 && r < nx - 1; // uniform per row
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float x0 = ring[base - t - 1][lane * C + c], xd = ring[base - t][lane * C + c];
                    const float t0 = x0 - (wvm[t][c] - wv0[t][c]);
                    const float t1 = xd - (wv0[t][c] - in[c]);
                    const float out = vd ? clip_to(fmaf(t1 - t0, inv_alpha, wv0[t][c]), T) : 0.0f;
                    wvm[t][c] = wv0[t][c];
                    wv0[t][c] = in[c];
                    in[c] = out;
                }
            }
            if (PB >= 0) continue; // the theta row is above the segment
            // row r = k - M + 1: final w_v in `in`; its horizontal iterations now
            const int r = k - M + 1;
            float xr[C], wh[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xr[c] = ring[base - M][lane * C + c];
                if constexpr (MODE == 1) wh[c] = hring.v[base - M][lane * C + c];
                else wh[c] = 0.0f;
            }
#pragma unroll
            for (int it = 0; it < M; ++it) {
                float t0[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float whl = c > 0 ? wh[c - 1] : from_left(wh[C - 1]);
                    t0[c] = xr[c] - (whl - wh[c]); // theta_h at this column
                }
                float nwh[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float t1 = c < C - 1 ? t0[c + 1] : from_right(t0[0]); // theta_h one column right
                    nwh[c] = hd[c] ? clip_to(fmaf(t1 - t0[c], inv_alpha, wh[c]), T) : 0.0f;
                }
#pragma unroll
                for (int c = 0; c < C; ++c) wh[c] = nwh[c];
            }
            float th[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float whl = c > 0 ? wh[c - 1] : from_left(wh[C - 1]);
                th[c] = theta_of(xr[c], whl, wh[c], cpm[c], in[c], 1.0f);
                cpm[c] = in[c];
            }
            if (r >= a && r < hi) { // uniform
                const uint32_t rowo = fo + (uint32_t)r * (uint32_t)ny;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if (!outc[c]) continue;
                    const uint32_t o = rowo + (uint32_t)(j0 + c);
                    if (theta_out) theta_out[o] = th[c];
                    if (u_out) u_out[o] = xr[c] - th[c];
                    if (w_out) {
                        w_out[o] = wh[c];
                        w_out[V + o] = in[c];
                    }
                }
            }
        }
    };
    static_for<0, NPRO>([&](auto pb) { chunk(decltype(pb)::value, pb); });
    for (int b = NPRO; b < nchunk; ++b) chunk(b, std::integral_constant<int, -1>{});
}

template <int M>
void launch_clip_m(int H, int nx, int ny, int B, const float *x, const float *w_in, float inv_alpha, float T,
                   float *w_out, float *theta, float *u_out, hipStream_t s)
{
    constexpr int C = kRowCols;
    constexpr int TXO = 64 * C - 2 * M - 1;
    const int nstrip = (ny + TXO - 1) / TXO, nseg = (nx + H - 1) / H;
    const dim3 g(nstrip * nseg * B), b(64);
    if (w_in)
        hipLaunchKernelGGL((k_clip_rows<M, C, 1>), g, b, 0, s, nx, ny, nstrip, nseg, H, x, w_in, inv_alpha, T, w_out,
                           theta, u_out);
    else
        hipLaunchKernelGGL((k_clip_rows<M, C, 0>), g, b, 0, s, nx, ny, nstrip, nseg, H, x, w_in, inv_alpha, T, w_out,
                           theta, u_out);
}

} // namespace

int launch_clip_rows(int H, int m, int nx, int ny, int B, const float *x, const float *w_in, float *w_out,
                     float alpha, float lambda, float *theta, float *u_out, hipStream_t s)
{
    const float ia = 1.0f / alpha, T = 2.0f * lambda;
    static_assert(kTileMaxM == 10, "pass lengths dispatched below");
    switch (m) {
#define SCI_M(mm)                                                                                                   \
    case mm: launch_clip_m<mm>(H, nx, ny, B, x, w_in, ia, T, w_out, theta, u_out, s); return SCI_OK;
        SCI_M(1) SCI_M(2) SCI_M(3) SCI_M(4) SCI_M(5) SCI_M(6) SCI_M(7) SCI_M(8) SCI_M(9) SCI_M(10)
#undef SCI_M
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
