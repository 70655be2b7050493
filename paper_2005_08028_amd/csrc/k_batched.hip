// Batched GAP-TV kernels: one launch covers every active problem of a batch
// of independent measurements with their own nx, ny and B.
//
// A device table of BatchProb descriptors holds, per problem, its sizes, its
// buffers and the first workgroup it owns in each kind of launch; a
// workgroup finds its problem by binary search over those prefix offsets
// (problems are sorted by descending outer-iteration count, so the active
// problems of outer iteration t are always a prefix of the table).
#include <hip/hip_runtime.h>

#include "k_fgp_rows.h"
#include "k_fgp_tile.h"
#include "k_fgp_tile_shapes.h"
#include "sci_batched.h"

namespace sci {
namespace {

constexpr int kPixBlock = 256;

// Largest p in [0, n) with base(p) <= w.
template <typename F>
__device__ inline int find_problem(int n, int w, F base)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base(mid) <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per problem: mask flag = 1 when it can be packed (B <= 32); cleared by the
// setup kernel on any entry that is neither 0 nor 1.
__global__ void k_batch_flags(int n, const BatchProb *__restrict__ tab)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p < n) *tab[p].cflag = tab[p].B <= 32 ? 1 : 0;
}

// theta^(0) = Phi^T y, Sinv = 1 / sum_k C_k^2 (0 where the sum is 0) and the
// masks packed one bit per frame.
__global__ __launch_bounds__(kPixBlock) void k_batch_setup(int n, const BatchProb *__restrict__ tab)
{
    const int p = find_problem(n, (int)blockIdx.x, [&](int q) { return tab[q].pb_base; });
    const BatchProb &b = tab[p];
    const uint32_t npix = (uint32_t)b.nx * (uint32_t)b.ny;
    const uint32_t pix = ((uint32_t)blockIdx.x - (uint32_t)b.pb_base) * kPixBlock + threadIdx.x;
    if (pix >= npix) return;
    const float y = b.Y[pix];
    float s = 0.0f;
    uint32_t bits = 0u;
    bool ok = true;
    for (int k = 0; k < b.B; ++k) {
        const uint32_t o = (uint32_t)k * npix + pix;
        const float c = b.C[o];
        s = fmaf(c, c, s);
        b.theta[o] = c * y;
        if (c == 1.0f) bits |= (k < 32 ? 1u << k : 0u);
        else if (c != 0.0f) ok = false;
    }
    s = s + 0.0f;
    b.Sinv[pix] = s > 0.0f ? 1.0f / s : 0.0f;
    b.cbits[pix] = bits;
    if (!ok) atomicAnd(b.cflag, 0);
}

// x = theta + C .* ((Y - sum_k C_k theta_k) .* Sinv), frames in registers.
// Problems flagged `pairs` take two adjacent pixels per thread (8-byte
// accesses, as the single-problem projection); the others one. The per-pixel
// arithmetic is the same either way.
template <int KB>
__device__ inline void batch_project_pair(const BatchProb &b, uint32_t q)
{
    const uint32_t npix = (uint32_t)b.nx * (uint32_t)b.ny;
    const uint32_t half = npix / 2; // float2 elements per frame
    if (q >= half) return;
    const int B = b.B;
    const bool packed = *b.cflag != 0;
    const uint2 m = packed ? ((const uint2 *)b.cbits)[q] : make_uint2(0u, 0u);
    const float2 *th = (const float2 *)b.theta, *C = (const float2 *)b.C;
    float2 v[KB], c[KB];
    float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * half + q;
            c[k] = packed ? make_float2((m.x >> k) & 1u ? 1.0f : 0.0f, (m.y >> k) & 1u ? 1.0f : 0.0f) : C[o];
            v[k] = th[o];
            acc0 = fmaf(c[k].x, v[k].x, acc0);
            acc1 = fmaf(c[k].y, v[k].y, acc1);
        }
    }
    const float2 yv = ((const float2 *)b.Y)[q], sv = ((const float2 *)b.Sinv)[q];
    const float r0 = (yv.x - acc0) * sv.x, r1 = (yv.y - acc1) * sv.y;
    float2 *x = (float2 *)b.x;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (k < B) x[(uint32_t)k * half + q] = make_float2(fmaf(c[k].x, r0, v[k].x), fmaf(c[k].y, r1, v[k].y));
}

template <int KB>
__global__ __launch_bounds__(kPixBlock) void k_batch_project(int n, const BatchProb *__restrict__ tab)
{
    const int p = find_problem(n, (int)blockIdx.x, [&](int q) { return tab[q].pj_base; });
    const BatchProb &b = tab[p];
    const uint32_t unit = ((uint32_t)blockIdx.x - (uint32_t)b.pj_base) * kPixBlock + threadIdx.x;
    if (b.pairs) { // uniform per workgroup
        batch_project_pair<KB>(b, unit);
        return;
    }
    const uint32_t npix = (uint32_t)b.nx * (uint32_t)b.ny;
    const uint32_t pix = unit;
    if (pix >= npix) return;
    const int B = b.B;
    const bool packed = *b.cflag != 0; // binary masks: one word of frame bits instead of B floats
    const uint32_t m = packed ? b.cbits[pix] : 0u;
    float v[KB], c[KB];
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < B) {
            const uint32_t o = (uint32_t)k * npix + pix;
            c[k] = packed ? ((m >> k) & 1u ? 1.0f : 0.0f) : b.C[o];
            v[k] = b.theta[o];
            acc = fmaf(c[k], v[k], acc);
        }
    }
    const float r = (b.Y[pix] - acc) * b.Sinv[pix];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (k < B) b.x[(uint32_t)k * npix + pix] = fmaf(c[k], r, v[k]);
}

// x = theta (problems that run no outer iteration).
__global__ __launch_bounds__(kPixBlock) void k_batch_copy_theta(int n, const BatchProb *__restrict__ tab)
{
    const int p = find_problem(n, (int)blockIdx.x, [&](int q) { return tab[q].pb_base; });
    const BatchProb &b = tab[p];
    const uint32_t npix = (uint32_t)b.nx * (uint32_t)b.ny;
    const uint32_t pix = ((uint32_t)blockIdx.x - (uint32_t)b.pb_base) * kPixBlock + threadIdx.x;
    if (pix >= npix || b.outer_iters != 0) return;
    for (int k = 0; k < b.B; ++k) b.x[(uint32_t)k * npix + pix] = b.theta[(uint32_t)k * npix + pix];
}

// theta = TVdenoise(x) from a zero dual, M iterations on chip, every tile of
// every frame of every active problem.
template <int TV, int M, int R, int NW, int C, int WPE>
__global__ __launch_bounds__(64 * NW, WPE) void k_batch_denoise(int n, const BatchProb *__restrict__ tab,
                                                                TileBeta bt, float lam, float step)
{
    __shared__ float lds_v[NW][64 * C];
    __shared__ float lds_t[NW][64 * C];
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int p = find_problem(n, lin, [&](int q) { return tab[q].wg_base; });
    const BatchProb &b = tab[p];
    const int local = lin - b.wg_base;
    const int frame = local / b.ntiles, tile = local % b.ntiles;
    const uint32_t plane = (uint32_t)b.nx * (uint32_t)b.ny;
    fgp_tile_body<TV, M, DT_F32, R, NW, C>(b.nx, b.ny, tile % b.ntx, tile / b.ntx, (uint32_t)frame * plane,
                                           plane * (uint32_t)b.B, b.x, nullptr, nullptr, 0, bt, lam, step, nullptr,
                                           nullptr, b.theta, nullptr, lds_v, lds_t);
}

// The same with the row-pipelined kernel: a one-wavefront workgroup per
// (strip, segment of H rows) of every frame of every active problem.
template <int TV, int M, int C>
__global__ __launch_bounds__(64, 2) void k_batch_rows(int n, const BatchProb *__restrict__ tab, TileBeta bt,
                                                      float lam, float step, int H)
{
    __shared__ RowRing<M, C> ring;
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int p = find_problem(n, lin, [&](int q) { return tab[q].wg_base; });
    const BatchProb &b = tab[p];
    const int local = lin - b.wg_base;
    const int frame = local / b.ntiles, tile = local % b.ntiles;
    const uint32_t plane = (uint32_t)b.nx * (uint32_t)b.ny;
    fgp_rows_body<TV, M, DT_F32, C, 0>(b.nx, b.ny, tile % b.ntx, tile / b.ntx, H, (uint32_t)frame * plane,
                                       plane * (uint32_t)b.B, b.x, nullptr, nullptr, bt, lam, step, nullptr, nullptr,
                                       b.theta, nullptr, ring);
}

template <int TV>
int launch_rows_batch(int H, int m, int n, int nwg, const BatchProb *tab, const TileBeta &bt, float lam,
                      hipStream_t s)
{
    const dim3 g(nwg), b(64);
    const float step = 1.0f / (8.0f * lam);
#define SCI_M(mm)                                                                                                   \
    case mm: hipLaunchKernelGGL((k_batch_rows<TV, mm, kRowCols>), g, b, 0, s, n, tab, bt, lam, step, H); return SCI_OK;
    switch (m) {
        SCI_M(1) SCI_M(2) SCI_M(3) SCI_M(4) SCI_M(5) SCI_M(6) SCI_M(7) SCI_M(8) SCI_M(9) SCI_M(10)
    }
#undef SCI_M
    return SCI_ERR_INVALID_ARG;
}

template <int TV, int R, int NW, int C, int WPE>
int launch_denoise_shape(int m, int n, int nwg, const BatchProb *tab, const TileBeta &bt, float lam, hipStream_t s)
{
    const dim3 g(nwg), b(64 * NW);
    const float step = 1.0f / (8.0f * lam);
#define SCI_M(mm)                                                                                                   \
    case mm: hipLaunchKernelGGL((k_batch_denoise<TV, mm, R, NW, C, WPE>), g, b, 0, s, n, tab, bt, lam, step); return SCI_OK;
    switch (m) {
        SCI_M(1) SCI_M(2) SCI_M(3) SCI_M(4) SCI_M(5) SCI_M(6) SCI_M(7) SCI_M(8) SCI_M(9) SCI_M(10)
    }
#undef SCI_M
    return SCI_ERR_INVALID_ARG;
}

template <int TV>
int launch_denoise_tv(int shape, int m, int n, int nwg, const BatchProb *tab, const TileBeta &bt, float lam,
                      hipStream_t s)
{
    switch (shape) {
#define SCI_CASE(id, R, NW, C, WPE)                                                                                 \
    case id: return launch_denoise_shape<TV, R, NW, C, WPE>(m, n, nwg, tab, bt, lam, s);
        SCI_TILE_SHAPES(SCI_CASE)
#undef SCI_CASE
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace

void batch_tile_extent(int shape, int m, int *tile_w, int *tile_h)
{
    int r = 0, w = 0, c = 0;
    tile_shape_info(shape, &r, &w, &c);
    *tile_w = 64 * c - 2 * m - 1;
    // a row-pipelined segment keeps all its rows; a tile loses its halo rows
    *tile_h = tile_shape_pipelined(shape) ? r : w * r - 2 * m - 1;
}

void launch_batch_setup(int n, int nblocks, const BatchProb *tab, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_flags, dim3((n + 255) / 256), dim3(256), 0, s, n, tab);
    hipLaunchKernelGGL(k_batch_setup, dim3(nblocks), dim3(kPixBlock), 0, s, n, tab);
    hipLaunchKernelGGL(k_batch_copy_theta, dim3(nblocks), dim3(kPixBlock), 0, s, n, tab);
}

int launch_batch_project(int n, int nblocks, int maxB, const BatchProb *tab, hipStream_t s)
{
    const dim3 g(nblocks), b(kPixBlock);
    if (maxB <= 8) hipLaunchKernelGGL(k_batch_project<8>, g, b, 0, s, n, tab);
    else if (maxB <= 16) hipLaunchKernelGGL(k_batch_project<16>, g, b, 0, s, n, tab);
    else if (maxB <= 32) hipLaunchKernelGGL(k_batch_project<32>, g, b, 0, s, n, tab);
    else return SCI_ERR_UNSUPPORTED;
    return SCI_OK;
}

int launch_batch_denoise(int tv, int shape, int m, int n, int nwg, const BatchProb *tab, const TileBeta &bt,
                         float lam, hipStream_t s)
{
    if (m < 1 || m > kTileMaxM) return SCI_ERR_INVALID_ARG;
    if (tile_shape_pipelined(shape)) {
        int H = 0, w = 0, c = 0;
        tile_shape_info(shape, &H, &w, &c);
        if (tv == TV_ATV) return launch_rows_batch<TV_ATV>(H, m, n, nwg, tab, bt, lam, s);
        if (tv == TV_ITV2D) return launch_rows_batch<TV_ITV2D>(H, m, n, nwg, tab, bt, lam, s);
        return SCI_ERR_UNSUPPORTED;
    }
    if (tv == TV_ATV) return launch_denoise_tv<TV_ATV>(shape, m, n, nwg, tab, bt, lam, s);
    if (tv == TV_ITV2D) return launch_denoise_tv<TV_ITV2D>(shape, m, n, nwg, tab, bt, lam, s);
    return SCI_ERR_UNSUPPORTED;
}

} // namespace sci
