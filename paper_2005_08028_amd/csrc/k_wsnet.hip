// Warm-start network kernels: a 4-layer 3x3x3 convolutional net over the
// (frame, row, column) volume that predicts the FGP dual field from the
// denoiser input, trained on (input, converged dual) pairs.
//
// Activations are channels-last bf16, [V][16] (V = B*nx*ny voxels, voxel
// v = (k*nx + i)*ny + j, 16 channels, unused channels zero). Weights are
// packed per layer as Wk[27][16 out][16 in] bf16 (tap t = (dk*3 + di)*3 + dj,
// offset (dk-1, di-1, dj-1)), with zero padding for the first layer's input
// channels and the last layer's output channels. The convolutions are
// implicit GEMMs on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the
// weights as the A operand, the staged input voxels as B; the mapping is
// described at the convolution kernel). The weight gradient runs on
// v_mfma_f32_16x16x16bf16_1k with the voxels as K.
//
// MFMA operand layouts (checked on the hardware): 16x16x16 - lane l holds A
// row l%16 and B column l%16 with K = 4*(l/16) .. +3; 16x16x32 - the same
// with K = 8*(l/16) .. +7; the result holds column l%16, rows
// 4*(l/16) .. +3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sci_internal.h"
#include "sci_math.h"
#include "sci_wsnet.h"

namespace sci {
namespace {

typedef short bf16x4 __attribute__((__vector_size__(4 * sizeof(short))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ inline uint16_t to_bf16(float v)
{
    uint32_t u = __float_as_uint(v);
    uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    if ((u & 0x7fffffffu) > 0x7f800000u) r = (u >> 16) | 0x40u;
    return (uint16_t)r;
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct Geom {
    int nx, ny, B;
    uint32_t V;
};

// ---- 3x3x3 convolution ------------------------------------------------------
//
// out[v][n] = sum_t sum_c Wk[t][n][c] in[nb(v, t)][c] + bias[n] over the
// volume, zero outside it ("same" padding). A workgroup owns a tile of
// kCI rows x kCJ columns and walks it through a run of frames; for output
// frame k it needs the input slabs (tile plus one-voxel halo) of frames
// k-1, k, k+1. Slabs sit in a ring of four in LDS: while frame k is computed
// from three of them, the fourth is free, and the global loads of the slab
// two frames ahead are in flight in registers. One barrier per frame.
//
// MFMA mapping (v_mfma_f32_16x16x32_bf16: A 16x32, B 32x16; lane l holds A
// row l%16 and B column l%16 with K = 8 (l/16) .. +7, and the result column
// l%16, rows 4 (l/16) .. +3). A row is an output voxel (16 consecutive
// columns of one output row), a result column an output channel. The K = 32
// of one instruction covers either two taps x 16 input channels or, for an
// input with at most 8 channels, four taps x 8 channels; taps are grouped by
// their (frame, column) offset (dk, dj), nine of them, so one operand read
// from staged row s serves output rows s, s-1, s-2 (di = 0, 1, 2) with the
// weights of (dk, di, dj): each wavefront computes four consecutive output
// rows from six staged rows and reads every operand once.
//
// The nine (dk, dj) offsets fill 5 (or 3) MFMAs with one (or three) K slots
// to spare; lanes of a spare slot read the last offset's data again and meet
// zero weights, so they add exact zeros, except that a non-finite staged
// value, which already turns the output it reaches into NaN or +-Inf through
// the real slot, makes it NaN.
//
// LDS layout: a staged voxel v (slab row si, column sj; v = si*kSJ + sj) is
// two 16-byte chunks (channels 0-7, 8-15); chunk h sits at slot
// 2v + (h xor (sj>>2 & 1)). Eight lanes reading chunk h of eight consecutive
// columns, or eight threads writing both chunks of four consecutive voxels,
// touch 32 distinct banks. An input with at most 8 channels stages one chunk
// per voxel, at slot v.
constexpr int kCI = 16, kCJ = 32;                     // output tile
constexpr int kSI = kCI + 2, kSJ = kCJ + 2;           // staged slab
constexpr int kSlabVox = kSI * kSJ;                   // 612 voxels
constexpr int kSlabChunks = 2 * kSlabVox;             // 1224 chunks, 19584 bytes
constexpr int kRing = 4;
constexpr int kChunkLoads = (kSlabChunks + 255) / 256; // per thread and slab, bf16 input
constexpr int kVoxLoads = (kSlabVox + 255) / 256;      // per thread and slab, fp32 input
constexpr int kRowsPerWave = kCI / 4;                  // 4 wavefronts

static_assert(kCJ == 32 && kRowsPerWave == 4, "the compute loop is written for 4 rows x 2 tiles per wavefront");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { CIN_BF16 = 0, CIN_F32 = 1 };          // input: bf16 [V][16], or fp32 planes x [V] (+ base [2][V])
enum { COUT_BF16 = 0, COUT_F32 = 1, COUT_DUAL = 2 };

struct ConvArgs {
    Geom g;
    int ntj, ntiles, F, nitems;  // tiles per row band, tiles per frame, frames per item, items
    const uint16_t *in;          // CIN_BF16
    const float *x, *xb0, *xb1;  // CIN_F32: x and the base planes (x itself when there is no base)
    int xb_live;                 // 0: channels 1, 2 are zero
    const uint16_t *Wk;
    const float *bias;           // nullable
    const uint16_t *gate;        // GATE: output zeroed where gate[v][n] <= 0
    uint16_t *out16;             // COUT_BF16: [V][16]
    float *out32;                // COUT_F32: [cout][V] raw; COUT_DUAL: [2][V] projected dual
    const float *obase;          // COUT_DUAL: base dual added before the projection (nullable)
    int cout, tv;                // COUT_F32 channels; COUT_DUAL: 0 ATV (clamp), 1 ITV2D (disc)
};

// two floats to bf16 (round to nearest even; v_cvt_pk_bf16_f32), packed low | high << 16
__device__ inline uint32_t pack2_bf16(float lo, float hi)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 p = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, p);
}

// Workgroups per CU: LDS holds two rings of 16-channel slabs, three of 8-channel ones.
template <int CIN> constexpr int conv_wgs_per_cu() { return CIN == CIN_F32 ? 3 : 2; }

template <int CIN, int COUT, bool RELU, bool GATE>
__global__ __launch_bounds__(256, conv_wgs_per_cu<CIN>()) void k_conv(const ConvArgs a)
{
    constexpr int CPT = CIN == CIN_F32 ? 1 : 2;   // chunks of a tap in one MFMA operand
    constexpr int TPM = 4 / CPT;                  // (dk, dj) offsets per MFMA
    constexpr int G = (9 + TPM - 1) / TPM;        // MFMAs per (staged row, di)
    constexpr int NL = CIN == CIN_F32 ? kVoxLoads : kChunkLoads;
    // LDS slot of chunk h of staged voxel v (slab column sj): one chunk per
    // voxel when only channels 0-7 are staged, else two, swizzled
    auto chunk_slot = [](int v, int sj, int h) { return CPT == 1 ? v : 2 * v + (h ^ ((sj >> 2) & 1)); };
    constexpr int SLAB = CPT == 1 ? kSlabVox : kSlabChunks; // 16-byte slots per slab
    __shared__ uint4 ring[kRing * SLAB];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int hsel = CPT == 2 ? (kq & 1) : 0;
    const int nx = a.g.nx, ny = a.g.ny, B = a.g.B;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny, V = a.g.V;

    // B operands: weights of tap (dk, di, dj) for the lane's (dk, dj) in group gi
    bf16x8 wb[3][G];
    int coff[G][2], cdk[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        const int c = TPM * gi + kq / CPT;
        const int cc = c < 9 ? c : 8, dk = cc / 3, dj = cc % 3;
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            if (c < 9) wb[di][gi] = *(const bf16x8 *)(a.Wk + ((size_t)(dk * 9 + di * 3 + dj) * 16 + row) * 16 + 8 * hsel);
            else wb[di][gi] = bf16x8{};
        }
        cdk[gi] = dk;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int col = 16 * tt + row + dj;
            coff[gi][tt] = chunk_slot(kRowsPerWave * wv * kSJ + col, col, hsel);
        }
    }
    float bn[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) bn[e] = a.bias ? a.bias[4 * kq + e] : 0.0f;

    // staging: this thread's chunks (bf16 input) or voxels (fp32 input) of a slab
    int pslot[NL];
    uint32_t poff[NL];
    uint32_t pok = 0;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
        const int e = tid + 256 * q;
        const int v = CIN == CIN_F32 ? e : (e >> 1), hh = CIN == CIN_F32 ? 0 : (e & 1);
        pslot[q] = chunk_slot(v, v % kSJ, hh);
    }
    uint4 pre[2][CIN == CIN_F32 ? 1 : NL];
    float px[2][CIN == CIN_F32 ? NL : 1], pb0[2][CIN == CIN_F32 ? NL : 1], pb1[2][CIN == CIN_F32 ? NL : 1];
    bool fval[2] = {false, false};

    auto q_live = [&](int q) { return q < NL - 1 || tid + 256 * q < (CIN == CIN_F32 ? kSlabVox : kSlabChunks); };

    // Every load is issued unconditionally (frames outside the volume read
    // the nearest frame, dead slots read offset 0) and the zeros are applied
    // when the slab is stored: with a fixed count of loads per slab the
    // wait for one slab's data lets the next slab's loads stay in flight.
    auto load_slab = [&](auto setc, int k0, int r) {
        constexpr int S = decltype(setc)::value;
        const int f = k0 - 1 + r;
        fval[S] = f >= 0 && f < B;
        const int fc = min(max(f, 0), B - 1);
        if constexpr (CIN == CIN_F32) {
            const size_t fb = (size_t)fc * plane;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                px[S][q] = a.x[fb + poff[q]];
                pb0[S][q] = a.xb0[fb + poff[q]];
                pb1[S][q] = a.xb1[fb + poff[q]];
            }
        } else {
            const uint16_t *src = a.in + (size_t)fc * plane * 16;
#pragma unroll
            for (int q = 0; q < NL; ++q) pre[S][q] = *(const uint4 *)(src + poff[q]);
        }
    };
    auto store_slab = [&](auto setc, int r) {
        constexpr int S = decltype(setc)::value;
        uint4 *slab = ring + (r & (kRing - 1)) * SLAB;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            if (!q_live(q)) continue;
            const bool ok = fval[S] && ((pok >> q) & 1u);
            uint4 val;
            if constexpr (CIN == CIN_F32)
                val = a.xb_live ? make_uint4(pack2_bf16(px[S][q], pb0[S][q]), pack2_bf16(pb1[S][q], 0.0f), 0u, 0u)
                                : make_uint4(pack2_bf16(px[S][q], 0.0f), 0u, 0u, 0u);
            else val = pre[S][q];
            slab[pslot[q]] = ok ? val : make_uint4(0u, 0u, 0u, 0u);
        }
    };

    const int nwg = (int)gridDim.x;
    for (int it = xcd_contiguous((int)blockIdx.x, nwg); it < a.nitems; it += nwg) {
        const int chunk = it / a.ntiles, tile = it % a.ntiles;
        const int i0 = (tile / a.ntj) * kCI, j0 = (tile % a.ntj) * kCJ, k0 = chunk * a.F;
        const int nf = min(a.F, B - k0);
        pok = 0;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + 256 * q;
            const int v = CIN == CIN_F32 ? e : (e >> 1), hh = CIN == CIN_F32 ? 0 : (e & 1);
            const int i = i0 - 1 + v / kSJ, j = j0 - 1 + v % kSJ;
            const bool ok = q_live(q) && i >= 0 && i < nx && j >= 0 && j < ny;
            poff[q] = ok ? (CIN == CIN_F32 ? (uint32_t)(i * ny + j) : (uint32_t)(i * ny + j) * 16u + 8u * hh) : 0u;
            pok |= (uint32_t)ok << q;
        }
        __syncthreads(); // every wavefront is done with the previous item's slabs
        load_slab(std::integral_constant<int, 0>{}, k0, 0);
        load_slab(std::integral_constant<int, 1>{}, k0, 1);
        store_slab(std::integral_constant<int, 0>{}, 0);
        store_slab(std::integral_constant<int, 1>{}, 1);
        load_slab(std::integral_constant<int, 0>{}, k0, 2);
        load_slab(std::integral_constant<int, 1>{}, k0, 3);

        auto step = [&](auto setc, int s) {
            store_slab(setc, s + 2);
            __syncthreads();
            const int k = k0 + s;
            const bool rows_live = i0 + kRowsPerWave * wv < nx; // uniform per wavefront
            // Loads complete in issue order: a kernel whose epilogue reads
            // memory (gate, base) requests those reads first and issues the
            // prefetch after the epilogue, so that waiting for them does not
            // wait for the prefetch.
            // Epilogue operands. The gate (GATE) is read before the compute
            // and the prefetch is issued after the epilogue: loads complete in
            // issue order, so waiting for the gate must not wait for a
            // prefetch. The base dual (COUT_DUAL) is read before the prefetch:
            // lane (row, kq) reads it for its own voxel of output row kq, and
            // the epilogue gathers it across lanes.
            uint2 eg[GATE ? 4 : 1][2];
            float eb[COUT == COUT_DUAL ? 2 : 1][2];
            if constexpr (GATE) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int tt = 0; tt < 2; ++tt) {
                        const int i = i0 + kRowsPerWave * wv + r, j = j0 + 16 * tt + row;
                        const size_t v = ((size_t)k * nx + i) * ny + j;
                        eg[r][tt] = i < nx && j < ny ? *(const uint2 *)(a.gate + v * 16 + 4 * kq) : make_uint2(0u, 0u);
                    }
            }
            if constexpr (COUT == COUT_DUAL) {
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    const int i = i0 + kRowsPerWave * wv + kq, j = j0 + 16 * tt + row;
                    const size_t v = ((size_t)k * nx + i) * ny + j;
                    const bool in = a.obase && i < nx && j < ny;
                    eb[tt][0] = in ? a.obase[v] : 0.0f;
                    eb[tt][1] = in ? a.obase[(size_t)V + v] : 0.0f;
                }
            }
            if constexpr (!GATE) load_slab(setc, k0, s + 4); // past the run's last slab: loaded, never stored
            if (rows_live) {
                // D[n][voxel] = sum_K W[n][K] X[K][voxel]: the weights are the
                // A operand, the staged voxels the B operand
                f32x4 acc[4][2];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int tt = 0; tt < 2; ++tt) acc[r][tt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                const uint4 *slab[G];
#pragma unroll
                for (int gi = 0; gi < G; ++gi) slab[gi] = ring + ((s + cdk[gi]) & (kRing - 1)) * SLAB;
                // (staged row u, group gi) in sequence; the operands of the
                // entry two ahead are read while the current one's MFMAs run
                constexpr int NP = (kRowsPerWave + 2) * G;
                bf16x8 X[3][2];
                auto rd = [&](int p, bf16x8(&b)[2]) {
                    const int u = p / G, gi = p % G;
#pragma unroll
                    for (int tt = 0; tt < 2; ++tt) b[tt] = __builtin_bit_cast(bf16x8, slab[gi][coff[gi][tt] + u * CPT * kSJ]);
                };
                rd(0, X[0]);
                rd(1, X[1]);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (p + 2 < NP) rd(p + 2, X[(p + 2) % 3]);
                    const int u = p / G, gi = p % G;
#pragma unroll
                    for (int di = 0; di < 3; ++di) {
                        const int r = u - di;
                        if (r < 0 || r >= kRowsPerWave) continue;
#pragma unroll
                        for (int tt = 0; tt < 2; ++tt)
                            acc[r][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[di][gi], X[p % 3][tt], acc[r][tt], 0, 0, 0);
                    }
                }

                // result: voxel j = j0 + 16 tt + row, output channels 4 kq + e
                float gb[COUT == COUT_DUAL ? 4 : 1][2][2];
                if constexpr (COUT == COUT_DUAL) {
                    // base of output row r: held by lane (row, r); every lane takes part
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
                                gb[r][tt][c] = __int_as_float(
                                    __builtin_amdgcn_ds_bpermute(4 * (row + 16 * r), __float_as_int(eb[tt][c])));
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + kRowsPerWave * wv + r;
                    if (i >= nx) break; // uniform per wavefront
                    const size_t vrow = ((size_t)k * nx + i) * ny;
#pragma unroll
                    for (int tt = 0; tt < 2; ++tt) {
                        const int j = j0 + 16 * tt + row;
                        if (j >= ny) continue;
                        const size_t v = vrow + j;
                        float y[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) y[e] = acc[r][tt][e] + bn[e];
                        if constexpr (COUT == COUT_DUAL) {
                            if (kq == 0) {
                                // (base +) output, entries with no difference 0, projected
                                float h = j < ny - 1 ? y[0] + gb[r][tt][0] : 0.0f;
                                float w = i < nx - 1 ? y[1] + gb[r][tt][1] : 0.0f;
                                if (a.tv == 0) {
                                    h = fminf(fmaxf(h, -1.0f), 1.0f);
                                    w = fminf(fmaxf(w, -1.0f), 1.0f);
                                } else {
                                    const float sc = fminf(1.0f, __builtin_amdgcn_rsqf(fmaf(w, w, h * h)));
                                    h *= sc;
                                    w *= sc;
                                }
                                a.out32[v] = h;
                                a.out32[(size_t)V + v] = w;
                            }
                        } else if constexpr (COUT == COUT_F32) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (4 * kq + e < a.cout) a.out32[(size_t)(4 * kq + e) * V + v] = y[e];
                        } else {
                            if (RELU)
#pragma unroll
                                for (int e = 0; e < 4; ++e) y[e] = fmaxf(y[e], 0.0f);
                            if constexpr (GATE) {
                                const uint2 gv = eg[r][tt];
                                if (!(__uint_as_float(gv.x << 16) > 0.0f)) y[0] = 0.0f;
                                if (!(__uint_as_float(gv.x & 0xffff0000u) > 0.0f)) y[1] = 0.0f;
                                if (!(__uint_as_float(gv.y << 16) > 0.0f)) y[2] = 0.0f;
                                if (!(__uint_as_float(gv.y & 0xffff0000u) > 0.0f)) y[3] = 0.0f;
                            }
                            *(uint2 *)(a.out16 + v * 16 + 4 * kq) = make_uint2(pack2_bf16(y[0], y[1]), pack2_bf16(y[2], y[3]));
                        }
                    }
                }
            }
            if constexpr (GATE) load_slab(setc, k0, s + 4);
        };
        // frames in pairs (both register sets on every trip, so the compiler
        // can count the loads in flight), then an odd last frame
        int s = 0;
        for (; s + 1 < nf; s += 2) {
            step(std::integral_constant<int, 0>{}, s);
            step(std::integral_constant<int, 1>{}, s + 1);
        }
        if (s < nf) step(std::integral_constant<int, 0>{}, s);
    }
}

// x [B][nx][ny] fp32 -> channels-last bf16 with x in channel 0 and, when
// given, a dual field [2][V] in channels 1 and 2.
__global__ __launch_bounds__(256) void k_pack_input(uint32_t V, const float *__restrict__ x,
                                                    const float *__restrict__ dual, uint16_t *__restrict__ a)
{
    const uint32_t v = blockIdx.x * 256u + threadIdx.x;
    if (v >= V) return;
    uint16_t *o = a + (size_t)v * 16;
    o[0] = to_bf16(x[v]);
    o[1] = dual ? to_bf16(dual[v]) : (uint16_t)0;
    o[2] = dual ? to_bf16(dual[V + v]) : (uint16_t)0;
#pragma unroll
    for (int c = 3; c < 16; ++c) o[c] = 0;
}

// Loss 1/(cout V) sum (y + base - target)^2 over the first cout channels
// (base: an optional [cout][V] field the output is added to), its gradient
// 2 (y + base - target) / (cout V) as bf16 [V][16] (other channels 0), and
// FP64 block partials of the squared error.
constexpr int kRedBlocks = 1024;
__global__ __launch_bounds__(256) void k_loss(uint32_t V, int cout, const float *__restrict__ y,
                                              const float *__restrict__ base, const float *__restrict__ target,
                                              uint16_t *__restrict__ dy, double *__restrict__ part)
{
    __shared__ double lds[256];
    const double scale = 2.0 / ((double)cout * (double)V);
    double acc = 0.0;
    for (uint32_t v = blockIdx.x * 256u + threadIdx.x; v < V; v += kRedBlocks * 256u) {
        uint16_t *o = dy + (size_t)v * 16;
        for (int c = 0; c < 16; ++c) {
            float gval = 0.0f;
            if (c < cout) {
                const double b = base ? (double)base[(size_t)c * V + v] : 0.0;
                const double d = ((double)y[(size_t)c * V + v] + b) - (double)target[(size_t)c * V + v];
                acc += d * d;
                gval = (float)(scale * d);
            }
            o[c] = to_bf16(gval);
        }
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

// theta-space loss (1/V) sum (D^T r)^2 with r = y + base - target on the two
// dual channels, entries that carry no difference (j = ny-1 for h, i = nx-1
// for v) held at 0 as D^T ignores them. The dual enters the denoiser's
// primal and its duality gap only through D^T p, so this loss ignores the
// components of the null space of D^T in which converged duals differ.
// Step 1: g = D^T r (float32 [V]) and FP64 block partials of sum g^2. The
// grid strides over columns (x), rows (y) and frames (z).
__device__ inline float r_h(const float *y, const float *base, const float *target, uint32_t V, uint32_t v, bool ex)
{
    if (!ex) return 0.0f;
    const float b = base ? base[v] : 0.0f;
    return (y[v] + b) - target[v];
}
__device__ inline float r_v(const float *y, const float *base, const float *target, uint32_t V, uint32_t v, bool ex)
{
    if (!ex) return 0.0f;
    const float b = base ? base[V + v] : 0.0f;
    return (y[V + v] + b) - target[V + v];
}

__global__ __launch_bounds__(256) void k_loss_theta_g(int nx, int ny, int B, const float *__restrict__ y,
                                                      const float *__restrict__ base,
                                                      const float *__restrict__ target, float *__restrict__ g,
                                                      double *__restrict__ part)
{
    __shared__ double lds[256];
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    double acc = 0.0;
    for (int k = (int)blockIdx.z; k < B; k += (int)gridDim.z)
        for (int i = (int)blockIdx.y; i < nx; i += (int)gridDim.y)
            for (int j = (int)blockIdx.x * 256 + (int)threadIdx.x; j < ny; j += (int)gridDim.x * 256) {
                const uint32_t v = (uint32_t)k * plane + (uint32_t)i * ny + (uint32_t)j;
                // (r_h(j-1) - r_h(j)) + (r_v(i-1) - r_v(i)), missing neighbours 0
                const float a = j >= 1 ? r_h(y, base, target, V, v - 1, true) : 0.0f;
                const float b = r_h(y, base, target, V, v, j < ny - 1);
                const float c = i >= 1 ? r_v(y, base, target, V, v - ny, true) : 0.0f;
                const float d = r_v(y, base, target, V, v, i < nx - 1);
                const float gv = (a - b) + (c - d);
                g[v] = gv;
                acc += (double)gv * (double)gv;
            }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = lds[0];
}

// Step 2: d loss / d y = (2/V) D g on the two dual channels (0 where the
// difference does not exist), as bf16 [V][16] with the other channels 0.
__global__ __launch_bounds__(256) void k_loss_theta_dy(int nx, int ny, int B, const float *__restrict__ g,
                                                       uint16_t *__restrict__ dy)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const float scale = (float)(2.0 / ((double)plane * (double)B));
    for (int k = (int)blockIdx.z; k < B; k += (int)gridDim.z)
        for (int i = (int)blockIdx.y; i < nx; i += (int)gridDim.y)
            for (int j = (int)blockIdx.x * 256 + (int)threadIdx.x; j < ny; j += (int)gridDim.x * 256) {
                const uint32_t v = (uint32_t)k * plane + (uint32_t)i * ny + (uint32_t)j;
                const float gc = g[v];
                const float dh = j < ny - 1 ? g[v + 1] - gc : 0.0f;
                const float dv = i < nx - 1 ? g[v + ny] - gc : 0.0f;
                uint16_t *o = dy + (size_t)v * 16;
                o[0] = to_bf16(scale * dh);
                o[1] = to_bf16(scale * dv);
#pragma unroll
                for (int c = 2; c < 16; ++c) o[c] = 0;
            }
}

__global__ __launch_bounds__(256) void k_sum_part(int n, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double lds[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) acc += part[b];
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

// Weight gradient dW[t][n][c] = sum_v dy[v][n] in[nb(v, t)][c] and
// dbias[n] = sum_v dy[v][n], as MFMAs with the voxels as K, over LDS blocks
// (the block shape of the convolution).
// A workgroup walks a fixed strided set of blocks; per block it stages the
// input with its halo and dy channel-major ([channel][voxel], bf16) so that
// the MFMA operands, whose K dimension runs over voxels, are runs of voxels
// of one channel. Wavefront w accumulates slots w, w+4, ... (27 taps and the
// bias) over 16-voxel chunks along j:
//   A[n][v'] = dy[v0 + v'][n]   (8-byte LDS read per lane)
//   B[v'][c] = in[nb(v0 + v', t)][c]   (four 2-byte LDS reads: a tap shifts
//   the run by dj, which breaks the 8-byte alignment)
// and writes its partial sums for the fixed-order reduction.
constexpr int kWgBlocks = 512;
constexpr int kTK = 4, kTI = 8, kTJ = 32;           // block of output voxels
constexpr int kHK = kTK + 2, kHI = kTI + 2, kHJ = kTJ + 2; // with its halo

__global__ __launch_bounds__(256) void k_wgrad_tile(Geom g, int ntj, int nti, int nblocks,
                                                    const uint16_t *__restrict__ dy, const uint16_t *__restrict__ in,
                                                    float *__restrict__ part)
{
    constexpr int NH = kHK * kHI * kHJ, NB = kTK * kTI * kTJ;
    __shared__ uint16_t xT[16][NH];
    __shared__ uint16_t dT[16][NB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    constexpr int kSlotsPerWave = 7; // 28 slots over 4 wavefronts
    f32x4 acc[kSlotsPerWave];
#pragma unroll
    for (int q = 0; q < kSlotsPerWave; ++q) acc[q] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    for (int blk = (int)blockIdx.x; blk < nblocks; blk += (int)gridDim.x) {
        const int bj = blk % ntj, bi = (blk / ntj) % nti, bk = blk / (ntj * nti);
        const int k0 = bk * kTK, i0 = bi * kTI, j0 = bj * kTJ;
        __syncthreads(); // the previous block's operands have been read
        for (int e = threadIdx.x; e < NH; e += 256) {
            const int jj = e % kHJ, ii = (e / kHJ) % kHI, kk = e / (kHJ * kHI);
            const int k = k0 + kk - 1, i = i0 + ii - 1, j = j0 + jj - 1;
            const bool ok = k >= 0 && k < g.B && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
            const uint16_t *src = in + (ok ? (((size_t)k * g.nx + i) * g.ny + j) * 16 : 0);
#pragma unroll
            for (int c = 0; c < 16; ++c) xT[c][e] = ok ? src[c] : (uint16_t)0;
        }
        for (int e = threadIdx.x; e < NB; e += 256) {
            const int jl = e % kTJ, il = (e / kTJ) % kTI, kl = e / (kTJ * kTI);
            const int k = k0 + kl, i = i0 + il, j = j0 + jl;
            const bool ok = k < g.B && i < g.nx && j < g.ny; // voxels outside the volume add nothing
            const uint16_t *src = dy + (ok ? (((size_t)k * g.nx + i) * g.ny + j) * 16 : 0);
#pragma unroll
            for (int n = 0; n < 16; ++n) dT[n][e] = ok ? src[n] : (uint16_t)0;
        }
        __syncthreads();
        for (int ch = 0; ch < NB / 16; ++ch) {
            const int kl = ch / (kTI * kTJ / 16), il = (ch / (kTJ / 16)) % kTI, jc = (ch % (kTJ / 16)) * 16;
            const int vb = (kl * kTI + il) * kTJ + jc; // first voxel of the chunk in the block
            const bf16x4 a = *(const bf16x4 *)(&dT[row][vb + 4 * kq]);
#pragma unroll
            for (int q = 0; q < kSlotsPerWave; ++q) {
                const int t = wv + 4 * q; // 0..27
                bf16x4 b;
                if (t == 27) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) b[e] = row == 0 ? (short)0x3f80 : (short)0; // bias: 1 in column 0
                } else {
                    const int dk = t / 9, di = (t / 3) % 3, dj = t % 3; // offsets into the haloed block
                    const int hb = ((kl + dk) * kHI + (il + di)) * kHJ + jc + dj + 4 * kq;
#pragma unroll
                    for (int e = 0; e < 4; ++e) b[e] = (short)xT[row][hb + e];
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
            }
        }
    }
    // acc[q]: column c = row, rows n = 4 kq + e
    float *p = part + (size_t)blockIdx.x * 28 * 256;
#pragma unroll
    for (int q = 0; q < kSlotsPerWave; ++q) {
        const int t = wv + 4 * q;
#pragma unroll
        for (int e = 0; e < 4; ++e) p[(size_t)t * 256 + (4 * kq + e) * 16 + row] = acc[q][e];
    }
}

// grad[t][n][c] = sum over groups in fixed order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(int ngroups, const float *__restrict__ part,
                                                      float *__restrict__ grad)
{
    const int idx = blockIdx.x * 256 + threadIdx.x; // 28 * 256 entries
    if (idx >= 28 * 256) return;
    float s = 0.0f;
    for (int b = 0; b < ngroups; ++b) s += part[(size_t)b * 28 * 256 + idx];
    grad[idx] = s;
}

// Adam on the fp32 master parameters of one layer in the padded layout
// [28][16][16] (slot 27 column 0 = bias); entries outside the layer's real
// channels stay zero. Then repack bf16 weights for the forward (Wk[t][n][c])
// and transposed (WkT[t'][c][n], t' = mirrored tap) convolutions.
__global__ __launch_bounds__(256) void k_adam(int cin, int cout, float lr, float b1, float b2, float eps, float c1,
                                              float c2, const float *__restrict__ grad, float *__restrict__ w,
                                              float *__restrict__ m, float *__restrict__ v,
                                              uint16_t *__restrict__ Wk, uint16_t *__restrict__ WkT,
                                              float *__restrict__ bias)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= 28 * 256) return;
    const int t = idx / 256, n = (idx / 16) % 16, c = idx % 16;
    const bool live = (t < 27) ? (n < cout && c < cin) : (n < cout && c == 0);
    if (live && lr != 0.0f) {
        const float gv = grad[idx];
        const float mm = b1 * m[idx] + (1.0f - b1) * gv;
        const float vv = b2 * v[idx] + (1.0f - b2) * gv * gv;
        m[idx] = mm;
        v[idx] = vv;
        w[idx] = w[idx] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
    const float wv = live ? w[idx] : 0.0f;
    if (t < 27) {
        Wk[(size_t)t * 256 + n * 16 + c] = to_bf16(wv);
        WkT[(size_t)(26 - t) * 256 + c * 16 + n] = to_bf16(wv);
    } else if (c == 0) {
        bias[n] = wv;
    }
}

// Network output [V][16] fp32 (channels 0, 1 = h, v), plus an optional base
// dual [2][V], -> dual [2][B][nx][ny] projected onto the TV's dual ball,
// entries with no difference zeroed.
__global__ __launch_bounds__(256) void k_dual_from_net(Geom g, int tv, const float *__restrict__ y,
                                                       const float *__restrict__ base, float *__restrict__ dual)
{
    const uint32_t pix = blockIdx.x * 256u + threadIdx.x;
    const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
    if (pix >= plane) return;
    const int i = (int)(pix / (uint32_t)g.ny), j = (int)(pix % (uint32_t)g.ny);
    const bool hin = j < g.ny - 1, vin = i < g.nx - 1;
    float n2 = 0.0f;
    if (tv == 2) {
        for (int k = 0; k < g.B; ++k) {
            const uint32_t v = (uint32_t)k * plane + pix;
            const float h = hin ? y[v] + (base ? base[v] : 0.0f) : 0.0f;
            const float w = vin ? y[g.V + v] + (base ? base[g.V + v] : 0.0f) : 0.0f;
            n2 = fmaf(w, w, fmaf(h, h, n2));
        }
    }
    const float svtv = fminf(1.0f, __builtin_amdgcn_rsqf(n2));
    for (int k = 0; k < g.B; ++k) {
        const uint32_t v = (uint32_t)k * plane + pix;
        float h = hin ? y[v] + (base ? base[v] : 0.0f) : 0.0f;
        float w = vin ? y[g.V + v] + (base ? base[g.V + v] : 0.0f) : 0.0f;
        if (tv == 0) {
            h = fminf(fmaxf(h, -1.0f), 1.0f);
            w = fminf(fmaxf(w, -1.0f), 1.0f);
        } else {
            const float s = tv == 1 ? fminf(1.0f, __builtin_amdgcn_rsqf(fmaf(w, w, h * h))) : svtv;
            h *= s;
            w *= s;
        }
        dual[v] = h;
        dual[g.V + v] = w;
    }
}

inline Geom geom(int nx, int ny, int B) { return Geom{nx, ny, B, (uint32_t)nx * ny * B}; }

} // namespace

void wsnet_pack_input(int nx, int ny, int B, const float *x, const float *dual, uint16_t *a, hipStream_t s)
{
    const uint32_t V = (uint32_t)nx * ny * B;
    hipLaunchKernelGGL(k_pack_input, dim3((V + 255) / 256), dim3(256), 0, s, V, x, dual, a);
}

namespace {

int device_cus()
{
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            ncu = n;
        else
            ncu = 256;
    }
    return ncu;
}

// Work split: tiles of kCI x kCJ, each walked through runs of F frames; the
// frames are cut into runs only when there are fewer tiles than resident
// workgroups (conv_wgs_per_cu per CU). Persistent grid of at most that many
// workgroups, each taking every gridDim-th item.
template <int CIN, int COUT, bool RELU, bool GATE>
void launch_conv(ConvArgs a, hipStream_t s)
{
    const int nti = (a.g.nx + kCI - 1) / kCI;
    a.ntj = (a.g.ny + kCJ - 1) / kCJ;
    a.ntiles = nti * a.ntj;
    const int slots = conv_wgs_per_cu<CIN>() * device_cus();
    const int runs = std::max(1, std::min(a.g.B, (slots + a.ntiles - 1) / a.ntiles));
    a.F = (a.g.B + runs - 1) / runs;
    a.nitems = a.ntiles * ((a.g.B + a.F - 1) / a.F);
    hipLaunchKernelGGL((k_conv<CIN, COUT, RELU, GATE>), dim3(std::min(a.nitems, slots)), dim3(256), 0, s, a);
}

ConvArgs conv_args(int nx, int ny, int B, const uint16_t *Wk, const float *bias)
{
    ConvArgs a{};
    a.g = geom(nx, ny, B);
    a.Wk = Wk;
    a.bias = bias;
    return a;
}

} // namespace

void wsnet_conv_input(int nx, int ny, int B, const float *x, const float *base, const uint16_t *Wk, const float *bias,
                      uint16_t *out16, hipStream_t s)
{
    ConvArgs a = conv_args(nx, ny, B, Wk, bias);
    const size_t V = (size_t)nx * ny * B;
    a.x = x;
    a.xb0 = base ? base : x;
    a.xb1 = base ? base + V : x;
    a.xb_live = base != nullptr;
    a.out16 = out16;
    launch_conv<CIN_F32, COUT_BF16, true, false>(a, s);
}

void wsnet_conv(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, bool relu,
                const uint16_t *gate, uint16_t *out16, hipStream_t s)
{
    ConvArgs a = conv_args(nx, ny, B, Wk, bias);
    a.in = in;
    a.gate = gate;
    a.out16 = out16;
    if (gate) launch_conv<CIN_BF16, COUT_BF16, false, true>(a, s);
    else if (relu) launch_conv<CIN_BF16, COUT_BF16, true, false>(a, s);
    else launch_conv<CIN_BF16, COUT_BF16, false, false>(a, s);
}

void wsnet_conv_out(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int cout,
                    float *y, hipStream_t s)
{
    ConvArgs a = conv_args(nx, ny, B, Wk, bias);
    a.in = in;
    a.out32 = y;
    a.cout = cout;
    launch_conv<CIN_BF16, COUT_F32, false, false>(a, s);
}

void wsnet_conv_dual(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int tv,
                     const float *base, float *dual, hipStream_t s)
{
    ConvArgs a = conv_args(nx, ny, B, Wk, bias);
    a.in = in;
    a.out32 = dual;
    a.obase = base;
    a.tv = tv;
    launch_conv<CIN_BF16, COUT_DUAL, false, false>(a, s);
}

int wsnet_reduce_blocks() { return kRedBlocks; }
int wsnet_wgrad_groups() { return kWgBlocks; }

void wsnet_loss(int nx, int ny, int B, int cout, const float *y, const float *base, const float *target, uint16_t *dy,
                double *part, double *out, hipStream_t s)
{
    const uint32_t V = (uint32_t)nx * ny * B;
    hipLaunchKernelGGL(k_loss, dim3(kRedBlocks), dim3(256), 0, s, V, cout, y, base, target, dy, part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, s, kRedBlocks, (const double *)part, out);
}

// Grid of the theta-loss kernels: column blocks x row strides x frame
// strides, at most kRedBlocks workgroups (the loss partials buffer).
dim3 theta_loss_grid(int nx, int ny, int B)
{
    const int gx = std::min((ny + 255) / 256, 16);
    const int gz = std::min(B, 8);
    const int gy = std::max(1, std::min(nx, kRedBlocks / (gx * gz)));
    return dim3(gx, gy, gz);
}

int wsnet_loss_theta(int nx, int ny, int B, const float *y, const float *base, const float *target, float *g,
                     uint16_t *dy, double *part, double *out, hipStream_t s)
{
    const dim3 grid = theta_loss_grid(nx, ny, B);
    const int nb = (int)(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL(k_loss_theta_g, grid, dim3(256), 0, s, nx, ny, B, y, base, target, g, part);
    hipLaunchKernelGGL(k_loss_theta_dy, grid, dim3(256), 0, s, nx, ny, B, (const float *)g, dy);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, s, nb, (const double *)part, out);
    return SCI_OK;
}

void wsnet_wgrad(int nx, int ny, int B, const uint16_t *dy, const uint16_t *in, float *part, float *grad,
                 hipStream_t s)
{
    const Geom g = geom(nx, ny, B);
    const int ntj = (ny + kTJ - 1) / kTJ, nti = (nx + kTI - 1) / kTI, ntk = (B + kTK - 1) / kTK;
    const int nblocks = ntj * nti * ntk;
    const int groups = nblocks < kWgBlocks ? nblocks : kWgBlocks;
    hipLaunchKernelGGL(k_wgrad_tile, dim3(groups), dim3(256), 0, s, g, ntj, nti, nblocks, dy, in, part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(28), dim3(256), 0, s, groups, (const float *)part, grad);
}

void wsnet_adam(int cin, int cout, float lr, float b1, float b2, float eps, float c1, float c2, const float *grad,
                float *w, float *m, float *v, uint16_t *Wk, uint16_t *WkT, float *bias, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(28), dim3(256), 0, s, cin, cout, lr, b1, b2, eps, c1, c2, grad, w, m, v, Wk, WkT,
                       bias);
}

void wsnet_dual_from_net(int nx, int ny, int B, int tv, const float *y, const float *base, float *dual, hipStream_t s)
{
    const Geom g = geom(nx, ny, B);
    const uint32_t plane = (uint32_t)nx * ny;
    hipLaunchKernelGGL(k_dual_from_net, dim3((plane + 255) / 256), dim3(256), 0, s, g, tv, y, base, dual);
}

} // namespace sci
