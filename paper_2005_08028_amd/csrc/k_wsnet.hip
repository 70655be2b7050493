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
// described at the convolution kernel). The weight gradient contracts over
// voxels on the same MFMA, its voxel-major operands taken from the LDS slab by
// transposing reads (ds_read_b64_tr_b16) and, for dy, made by
// v_mfma_f32_16x16x16bf16_1k against the identity.
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

struct Geom {
    int nx, ny, B;
    uint32_t V;
};

// ---- 3x3x3 convolution ------------------------------------------------------
//
// out[v][n] = sum_t sum_c Wk[t][n][c] in[nb(v, t)][c] + bias[n] over the
// volume, zero outside it ("same" padding). A workgroup owns a tile of
// 4 x (wavefronts) rows x kCJ columns and walks it through a run of frames;
// for output frame k it needs the input slabs (tile plus one-voxel halo) of
// frames k-1, k, k+1, held in a ring in LDS while the global loads of the
// slab two frames ahead are in flight in registers (WalkShape).
//
// MFMA mapping (v_mfma_f32_16x16x32_bf16: A 16x32, B 32x16; lane l holds A
// row l%16 and B column l%16 with K = 8 (l/16) .. +7, and the result column
// l%16, rows 4 (l/16) .. +3). The weights are A (a row is an output
// channel), the staged input B (a column is an output voxel, one of 16
// consecutive columns of an output row), so a lane's result is four output
// channels of one voxel. The K = 32 of one instruction covers either two
// taps x 16 input channels or, for an input with at most 8 channels, four
// taps x 8 channels; taps are grouped by their (frame, column) offset
// (dk, dj), nine of them, so one operand read from staged row s serves output
// rows s, s-1, s-2 (di = 0, 1, 2) with the weights of (dk, di, dj): each
// wavefront computes four consecutive output rows from six staged rows and
// reads every operand once.
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
constexpr int kRowsPerWave = 4, kCJ = 32;             // output rows per wavefront, tile columns
constexpr int kSJ = kCJ + 2;                          // staged slab columns

// Tile, slab and pipelining of a frame walk by workgroups of NW wavefronts:
// NW * 4 output rows per tile. With several wavefronts the ring holds four
// slabs (the one written at a step start was last read two steps before, and
// the step's barrier orders that read before the write) and two register
// sets of slabs are in flight; a lone wavefront reads and writes its LDS in
// program order, so three slabs and one register set suffice.
template <int NW, int RG = NW> struct WalkShape { // RG groups of 4 rows
    static constexpr int NT = 64 * NW;
    static constexpr int CI = kRowsPerWave * RG;
    static constexpr int VOX = (CI + 2) * kSJ; // staged voxels per slab
    static constexpr int RING = NW == 1 ? 3 : 4;
    static constexpr int SETS = NW == 1 ? 1 : 2;
    __device__ static int slot(int r) { return RING == 4 ? (r & 3) : (r % 3); }
};

static_assert(kCJ == 32 && kRowsPerWave == 4, "the compute loop is written for 4 rows x 2 tiles per wavefront");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { CIN_BF16 = 0, CIN_F32 = 1 };          // input: bf16 [V][16], or fp32 planes x [V] (+ base [2][V])
enum { COUT_BF16 = 0, COUT_F32 = 1, COUT_DUAL = 2 };

// Where a frame walk takes its input from.
struct SlabSrc {
    const uint16_t *in;          // CIN_BF16: [V][16]
    const float *x, *xb0, *xb1;  // CIN_F32: x and the base planes (x itself when there is no base)
    int xb_live;                 // 0: channels 1, 2 are zero
};

// Tiles, frame runs and items of a frame walk.
struct WalkGeom {
    Geom g;
    int ntj, ntiles, F, nitems;  // tiles per row band, tiles per frame, frames per run, items
};

struct ConvArgs {
    WalkGeom w;
    SlabSrc src;
    const uint16_t *Wk;
    const float *bias;           // nullable
    const uint8_t *gate;         // GATE: sign bytes [V][4] (bit e of byte q: channel 4q+e > 0); output zeroed where clear
    uint16_t *out16;             // COUT_BF16: [V][16]
    uint8_t *sign;               // COUT_BF16 (nullable): sign bytes of the bf16 output, layout as gate
    float *out32;                // COUT_F32: [cout][V] raw; COUT_DUAL: [2][V] projected dual
    const float *obase;          // COUT_DUAL: base dual added before the projection (nullable)
    int cout, tv;                // output channels (2 for COUT_DUAL); COUT_DUAL: 0 ATV (clamp), 1 ITV2D (disc)
};

// per-lane choice without a branch: a where mask is all ones, b where it is 0
__device__ inline float pick(uint32_t mask, float a, float b)
{
    return __uint_as_float((__float_as_uint(a) & mask) | (__float_as_uint(b) & ~mask));
}

// two floats to bf16 (round to nearest even; v_cvt_pk_bf16_f32), packed low | high << 16
__device__ inline uint32_t pack2_bf16(float lo, float hi)
{
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 p = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, p);
}

// Staging of input slabs (tile plus halo, one frame) through registers into
// the LDS ring. Each thread owns NL fixed slots of a slab; two register sets
// hold the slabs in flight.
template <int CIN, int NW, int RG = NW> struct SlabStage {
    using W = WalkShape<NW, RG>;
    static constexpr int CPT = CIN == CIN_F32 ? 1 : 2;  // 16-byte chunks per staged voxel
    static constexpr int SLAB = CPT * W::VOX;           // 16-byte slots per slab
    static constexpr int NL = (SLAB + W::NT - 1) / W::NT; // slots per thread
    static constexpr int S = W::SETS;

    // LDS slot of chunk h of staged voxel v (slab column sj): one chunk per
    // voxel when only channels 0-7 are staged, else two, swizzled
    __device__ static int chunk_slot(int v, int sj, int h) { return CPT == 1 ? v : 2 * v + (h ^ ((sj >> 2) & 1)); }
    // 8-byte LDS index of quarter q (channels 4q .. 4q+3) of staged voxel v
    __device__ static int quarter_slot(int v, int sj, int q) { return 2 * chunk_slot(v, sj, q >> 1) + (q & 1); }

    int pslot[NL];
    uint32_t poff[NL];
    uint32_t pok;
    uint4 pre[S][CIN == CIN_F32 ? 1 : NL];
    float px[S][CIN == CIN_F32 ? NL : 1], pb0[S][CIN == CIN_F32 ? NL : 1], pb1[S][CIN == CIN_F32 ? NL : 1];
    bool fval[S];

    __device__ static bool live(int tid, int q) { return q < NL - 1 || tid + W::NT * q < SLAB; }
    __device__ static void split(int e, int &v, int &hh)
    {
        v = CIN == CIN_F32 ? e : (e >> 1);
        hh = CIN == CIN_F32 ? 0 : (e & 1);
    }

    __device__ void init(int tid)
    {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            int v, hh;
            split(tid + W::NT * q, v, hh);
            pslot[q] = chunk_slot(v, v % kSJ, hh);
        }
#pragma unroll
        for (int k = 0; k < S; ++k) fval[k] = false;
    }
    // source offsets within a frame for the tile at (i0, j0); zero outside the frame
    __device__ void begin(int tid, int i0, int j0, int nx, int ny)
    {
        pok = 0;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            int v, hh;
            split(tid + W::NT * q, v, hh);
            const int i = i0 - 1 + v / kSJ, j = j0 - 1 + v % kSJ;
            const bool ok = live(tid, q) && i >= 0 && i < nx && j >= 0 && j < ny;
            poff[q] = ok ? (CIN == CIN_F32 ? (uint32_t)(i * ny + j) : (uint32_t)(i * ny + j) * 16u + 8u * hh) : 0u;
            pok |= (uint32_t)ok << q;
        }
    }
    // Every load is issued unconditionally (a frame outside the volume reads
    // the nearest frame, dead slots read offset 0) and the zeros are applied
    // when the slab is stored: with a fixed count of loads per slab, the wait
    // for one slab's data lets the next slab's loads stay in flight.
    template <int K> __device__ void load(const SlabSrc &src, const Geom &g, int f)
    {
        fval[K] = f >= 0 && f < g.B;
        const int fc = min(max(f, 0), g.B - 1);
        const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
        if constexpr (CIN == CIN_F32) {
            const size_t fb = (size_t)fc * plane;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                px[K][q] = src.x[fb + poff[q]];
                pb0[K][q] = src.xb0[fb + poff[q]];
                pb1[K][q] = src.xb1[fb + poff[q]];
            }
        } else {
            const uint16_t *p = src.in + (size_t)fc * plane * 16;
#pragma unroll
            for (int q = 0; q < NL; ++q) pre[K][q] = *(const uint4 *)(p + poff[q]);
        }
    }
    template <int K> __device__ void store(const SlabSrc &src, uint4 *slab, int tid)
    {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            if (!live(tid, q)) continue;
            const bool ok = fval[K] && ((pok >> q) & 1u);
            uint4 val;
            if constexpr (CIN == CIN_F32)
                val = src.xb_live ? make_uint4(pack2_bf16(px[K][q], pb0[K][q]), pack2_bf16(pb1[K][q], 0.0f), 0u, 0u)
                                  : make_uint4(pack2_bf16(px[K][q], 0.0f), 0u, 0u, 0u);
            else val = pre[K][q];
            slab[pslot[q]] = ok ? val : make_uint4(0u, 0u, 0u, 0u);
        }
    }
};

// The frame walk: this workgroup's items (tile, run of frames), every
// gridDim-th item after an XCD-contiguous renumbering. For output frame k0 + s
// of an item, slabs r = s, s+1, s+2 (frames k0-1+r) are in LDS ring slots
// W::slot(r); step(setc, s, i0, j0, k, prefetch) computes it and must call
// prefetch() exactly once (uniformly), which issues the loads of slab
// s + 2 + SETS into the register set the step's store has just emptied.
// begin(i0, j0, k0) runs once per item, after the first slabs are requested.
template <typename St, typename Step, typename Begin>
__device__ __forceinline__ void frame_walk(const WalkGeom &w, const SlabSrc &src, uint4 *ring, St &st, Step &&step,
                                           Begin &&begin)
{
    using W = typename St::W;
    const int tid = threadIdx.x, nwg = (int)gridDim.x;
    auto slab = [&](int r) { return ring + W::slot(r) * St::SLAB; };
    for (int it = xcd_contiguous((int)blockIdx.x, nwg); it < w.nitems; it += nwg) {
        const int run = it / w.ntiles, tile = it % w.ntiles;
        const int i0 = (tile / w.ntj) * W::CI, j0 = (tile % w.ntj) * kCJ, k0 = run * w.F;
        const int nf = min(w.F, w.g.B - k0);
        st.begin(tid, i0, j0, w.g.nx, w.g.ny);
        __syncthreads(); // every wavefront is done with the previous item's slabs
        if constexpr (W::SETS == 2) {
            st.template load<0>(src, w.g, k0 - 1);
            st.template load<1>(src, w.g, k0);
            st.template store<0>(src, slab(0), tid);
            st.template store<1>(src, slab(1), tid);
            st.template load<0>(src, w.g, k0 + 1);
            st.template load<1>(src, w.g, k0 + 2);
        } else {
            st.template load<0>(src, w.g, k0 - 1);
            st.template store<0>(src, slab(0), tid);
            st.template load<0>(src, w.g, k0);
            st.template store<0>(src, slab(1), tid);
            st.template load<0>(src, w.g, k0 + 1);
        }
        begin(i0, j0, k0);
        auto one = [&](auto setc, int s) {
            constexpr int K = decltype(setc)::value;
            st.template store<K>(src, slab(s + 2), tid);
            __syncthreads();
            // past the run's last slab: loaded, never stored
            auto prefetch = [&] { st.template load<K>(src, w.g, k0 + s + 1 + W::SETS); };
            step(setc, s, i0, j0, k0 + s, prefetch);
        };
        int s = 0;
        if constexpr (W::SETS == 2) {
            // frames in pairs (both register sets on every trip, so the
            // compiler can count the loads in flight), then an odd last frame
            for (; s + 1 < nf; s += 2) {
                one(std::integral_constant<int, 0>{}, s);
                one(std::integral_constant<int, 1>{}, s + 1);
            }
            if (s < nf) one(std::integral_constant<int, 0>{}, s);
        } else {
            for (; s < nf; ++s) one(std::integral_constant<int, 0>{}, s);
        }
    }
}

// The convolutions run 4-wavefront workgroups, two wavefronts per SIMD (the
// LDS of two 16-channel rings per CU; registers), three for the 8-channel
// first layer. (One-wavefront workgroups, eight per CU with a 3-slab ring
// each and no barrier, measured no faster: 350-475 against 340-470 us for a
// hidden layer at 1024x1024x24, and the first layer 15-25 % slower.)
constexpr int kConvNW = 4;
template <int CIN> constexpr int conv_waves_per_simd() { return CIN == CIN_F32 ? 3 : 2; }
template <int CIN> constexpr int conv_wgs_per_cu() { return conv_waves_per_simd<CIN>() * 4 / kConvNW; }

// PACK (an output of at most 4 channels): row m = 4 di + n of the weight
// operand holds output channel n at row offset di, so one MFMA applies all
// three row offsets to a staged row. Its result for staged row u, row m, is
// then a partial sum of output row u - di, and output row r is the sum of the
// partials of staged rows r, r+1, r+2 (lane groups kq = 0, 1, 2): a
// reduce-scatter across the lane groups (ds_bpermute) leaves lane (column, kq)
// with output row kq. Half the MFMAs of the 16-channel mapping, and the
// epilogue runs on all 64 lanes.
template <int CIN, int COUT, bool RELU, bool GATE, bool PACK = false>
__global__ __launch_bounds__(64 * kConvNW, conv_waves_per_simd<CIN>()) void k_conv(const ConvArgs a)
{
    using St = SlabStage<CIN, kConvNW>;
    using W = WalkShape<kConvNW>;
    constexpr int CPT = St::CPT;                  // chunks of a tap in one MFMA operand
    constexpr int TPM = 4 / CPT;                  // (dk, dj) offsets per MFMA
    constexpr int G = (9 + TPM - 1) / TPM;        // MFMAs per (staged row, di)
    static_assert(!PACK || (CIN == CIN_BF16 && COUT != COUT_BF16), "packed rows: a 16-channel input, fp32 output");
    static_assert(COUT != COUT_DUAL || PACK, "the dual output is packed");
    __shared__ uint4 ring[W::RING * St::SLAB];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int hsel = CPT == 2 ? (kq & 1) : 0;
    const int nx = a.w.g.nx, ny = a.w.g.ny;
    const uint32_t V = a.w.g.V;

    // A operands: weights of tap (dk, di, dj) for the lane's (dk, dj) in group gi
    // (PACK: di and the output channel from the row)
    bf16x8 wb[PACK ? 1 : 3][G];
    int coff[G][2], cdk[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        const int c = TPM * gi + kq / CPT;
        const int cc = c < 9 ? c : 8, dk = cc / 3, dj = cc % 3;
        if constexpr (PACK) {
            const int di = row >> 2, n = row & 3;
            wb[0][gi] = c < 9 && di < 3 && n < a.cout
                            ? *(const bf16x8 *)(a.Wk + ((size_t)(dk * 9 + di * 3 + dj) * 16 + n) * 16 + 8 * hsel)
                            : bf16x8{};
        } else {
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                if (c < 9) wb[di][gi] = *(const bf16x8 *)(a.Wk + ((size_t)(dk * 9 + di * 3 + dj) * 16 + row) * 16 + 8 * hsel);
                else wb[di][gi] = bf16x8{};
            }
        }
        cdk[gi] = dk;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int col = 16 * tt + row + dj;
            coff[gi][tt] = St::chunk_slot(kRowsPerWave * wv * kSJ + col, col, hsel);
        }
    }
    float bn[4]; // PACK: bias of channel e; else of channel 4 kq + e
#pragma unroll
    for (int e = 0; e < 4; ++e) bn[e] = a.bias ? a.bias[PACK ? e : 4 * kq + e] : 0.0f;

    // The epilogue's operands at the lane's own voxel of output row kq, set
    // S of frame k: the base dual (COUT_DUAL), the four sign bytes (GATE;
    // the epilogue takes row r's from lane (row, r)). With two register sets
    // they are read a frame ahead, before the slab prefetch, so that the wait
    // for them does not wait for a slab.
    float eb[2][2][2];
    uint32_t egw[2][2];
    auto load_epi = [&](auto setc, int i0, int j0, int k) {
        constexpr int S = decltype(setc)::value;
        const int kc = min(k, a.w.g.B - 1); // past the last frame: read, never used
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int i = i0 + kRowsPerWave * wv + kq, j = j0 + 16 * tt + row;
            const size_t v = ((size_t)kc * nx + i) * ny + j;
            if constexpr (COUT == COUT_DUAL) {
                const bool in = a.obase && i < nx && j < ny;
                eb[S][tt][0] = in ? a.obase[v] : 0.0f;
                eb[S][tt][1] = in ? a.obase[(size_t)V + v] : 0.0f;
            }
            if constexpr (GATE) egw[S][tt] = i < nx && j < ny ? *(const uint32_t *)(a.gate + v * 4) : 0u;
        }
    };
    constexpr bool EPI = COUT == COUT_DUAL || GATE;
    constexpr bool AHEAD = EPI && W::SETS == 2;

    St st;
    st.init(tid);
    frame_walk(a.w, a.src, ring, st, [&](auto setc, int s, int i0, int j0, int k, auto &&prefetch) {
        constexpr int S = AHEAD ? decltype(setc)::value : 0;
        const bool rows_live = i0 + kRowsPerWave * wv < nx; // uniform per wavefront
        // With one register set the loads of the slab two frames ahead go out
        // first: they have this step's compute to arrive.
        if constexpr (W::SETS == 1) prefetch();
        // Vector memory operations complete in issue order, and the
        // epilogue's stores are conditional, so the compiler cannot count
        // them: the prefetch is issued after the epilogue, and the wait for
        // a slab (two steps later) then leaves the next slab's loads in
        // flight.
        if constexpr (EPI && !AHEAD) load_epi(std::integral_constant<int, 0>{}, i0, j0, k);
        if (rows_live) {
            // D[n][voxel] = sum_K W[n][K] X[K][voxel]: the weights are the
            // A operand, the staged voxels the B operand. acc[q][tt]: output
            // row q, or (PACK) the partials of staged row q.
            constexpr int NQ = PACK ? kRowsPerWave + 2 : kRowsPerWave;
            f32x4 acc[NQ][2];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) acc[q][tt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            const uint4 *slab[G];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) slab[gi] = ring + W::slot(s + cdk[gi]) * St::SLAB;
            // (staged row u, group gi) in sequence, u inner for PACK (so
            // that consecutive MFMAs feed different accumulators); the
            // operands of the entry two ahead are read while the current
            // one's MFMAs run
            constexpr int NU = kRowsPerWave + 2, NP = NU * G;
            auto entry = [](int p, int &u, int &gi) {
                u = PACK ? p % NU : p / G;
                gi = PACK ? p / NU : p % G;
            };
            bf16x8 X[3][2];
            auto rd = [&](int p, bf16x8(&b)[2]) {
                int u, gi;
                entry(p, u, gi);
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) b[tt] = __builtin_bit_cast(bf16x8, slab[gi][coff[gi][tt] + u * CPT * kSJ]);
            };
            // interleave the LDS reads with the MFMAs (the compiler's
            // small-GEMM schedule; the 8-channel first layer would spill)
            if constexpr (CPT == 2) __builtin_amdgcn_iglp_opt(0);
            rd(0, X[0]);
            rd(1, X[1]);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (p + 2 < NP) rd(p + 2, X[(p + 2) % 3]);
                int u, gi;
                entry(p, u, gi);
                if constexpr (PACK) {
#pragma unroll
                    for (int tt = 0; tt < 2; ++tt)
                        acc[u][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[0][gi], X[p % 3][tt], acc[u][tt], 0, 0, 0);
                } else {
#pragma unroll
                    for (int di = 0; di < 3; ++di) {
                        const int r = u - di;
                        if (r < 0 || r >= kRowsPerWave) continue;
#pragma unroll
                        for (int tt = 0; tt < 2; ++tt)
                            acc[r][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[di][gi], X[p % 3][tt], acc[r][tt], 0, 0, 0);
                    }
                }
            }

            if constexpr (PACK) {
                // lane (row, kq) holds partial (di = kq, channel e) of staged
                // row q in acc[q][tt][e]; t[r] = its share of output row r
                // (group 3 holds none). Reduce-scatter: lane groups kq and
                // kq ^ 2 add the rows of their half (rows 2h, 2h+1, h = kq>>1),
                // then kq and kq ^ 1 add row kq.
                constexpr int NE = COUT == COUT_DUAL ? 2 : 4; // channels reduced
                const uint32_t g0 = 0u - (uint32_t)(kq == 0), g1 = 0u - (uint32_t)(kq == 1),
                               g2 = 0u - (uint32_t)(kq == 2);
                const uint32_t mh = 0u - (uint32_t)(kq >> 1), mb = 0u - (uint32_t)(kq & 1);
                const int up = 4 * (lane ^ 32), side = 4 * (lane ^ 16);
                float y[NE][2];
#pragma unroll
                for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                    for (int e = 0; e < NE; ++e) {
                        float t[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            t[r] = pick(g0, acc[r][tt][e], pick(g1, acc[r + 1][tt][e], pick(g2, acc[r + 2][tt][e], 0.0f)));
                        const float s0 = pick(mh, t[0], t[2]), s1 = pick(mh, t[1], t[3]);
                        const float a0 = pick(mh, t[2], t[0]) + __int_as_float(__builtin_amdgcn_ds_bpermute(up, __float_as_int(s0)));
                        const float a1 = pick(mh, t[3], t[1]) + __int_as_float(__builtin_amdgcn_ds_bpermute(up, __float_as_int(s1)));
                        const float snd = pick(mb, a0, a1);
                        y[e][tt] = pick(mb, a1, a0) + __int_as_float(__builtin_amdgcn_ds_bpermute(side, __float_as_int(snd)));
                    }
                // lane (row, kq): output row kq, column j0 + 16 tt + row
                const int i = i0 + kRowsPerWave * wv + kq;
#pragma unroll
                for (int tt = 0; tt < 2; ++tt) {
                    const int j = j0 + 16 * tt + row;
                    if (i >= nx || j >= ny) continue;
                    const size_t v = ((size_t)k * nx + i) * ny + j;
                    if constexpr (COUT == COUT_DUAL) {
                        // (base +) output, entries with no difference 0, projected
                        float hh = j < ny - 1 ? (y[0][tt] + bn[0]) + eb[S][tt][0] : 0.0f;
                        float ww = i < nx - 1 ? (y[1][tt] + bn[1]) + eb[S][tt][1] : 0.0f;
                        if (a.tv == 0) {
                            hh = fminf(fmaxf(hh, -1.0f), 1.0f);
                            ww = fminf(fmaxf(ww, -1.0f), 1.0f);
                        } else {
                            const float sc = fminf(1.0f, __builtin_amdgcn_rsqf(fmaf(ww, ww, hh * hh)));
                            hh *= sc;
                            ww *= sc;
                        }
                        a.out32[v] = hh;
                        a.out32[(size_t)V + v] = ww;
                    } else {
#pragma unroll
                        for (int e = 0; e < NE; ++e)
                            if (e < a.cout) a.out32[(size_t)e * V + v] = y[e][tt] + bn[e];
                    }
                }
            } else {
                // result: voxel j = j0 + 16 tt + row, output channels 4 kq + e
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
                        if constexpr (COUT == COUT_F32) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (4 * kq + e < a.cout) a.out32[(size_t)(4 * kq + e) * V + v] = y[e];
                        } else {
                            if (RELU)
#pragma unroll
                                for (int e = 0; e < 4; ++e) y[e] = fmaxf(y[e], 0.0f);
                            if constexpr (GATE) {
                                const uint32_t gw =
                                    (uint32_t)__builtin_amdgcn_ds_bpermute(4 * (row + 16 * r), (int)egw[S][tt]);
                                const uint32_t gb = gw >> (8 * kq);
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    if (!((gb >> e) & 1u)) y[e] = 0.0f;
                            }
                            const uint2 o = make_uint2(pack2_bf16(y[0], y[1]), pack2_bf16(y[2], y[3]));
                            *(uint2 *)(a.out16 + v * 16 + 4 * kq) = o;
                            if (a.sign) // uniform
                                a.sign[v * 4 + kq] = (uint8_t)((__uint_as_float(o.x << 16) > 0.0f) |
                                                               (__uint_as_float(o.x & 0xffff0000u) > 0.0f) << 1 |
                                                               (__uint_as_float(o.y << 16) > 0.0f) << 2 |
                                                               (__uint_as_float(o.y & 0xffff0000u) > 0.0f) << 3);
                        }
                    }
                }
            }
        }
        if constexpr (W::SETS == 2) {
            if constexpr (AHEAD) load_epi(std::integral_constant<int, 1 - S>{}, i0, j0, k + 1);
            prefetch();
        }
    }, [&](int i0, int j0, int k0) {
        if constexpr (AHEAD) load_epi(std::integral_constant<int, 0>{}, i0, j0, k0);
    });
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
        uint32_t w[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c >= cout) break;
            const double b = base ? (double)base[(size_t)c * V + v] : 0.0;
            const double d = ((double)y[(size_t)c * V + v] + b) - (double)target[(size_t)c * V + v];
            acc += d * d;
            w[c >> 1] |= (uint32_t)to_bf16((float)(scale * d)) << (16 * (c & 1));
        }
        uint4 *o = (uint4 *)(dy + (size_t)v * 16);
        o[0] = make_uint4(w[0], w[1], w[2], w[3]);
        o[1] = make_uint4(w[4], w[5], w[6], w[7]);
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
                uint4 *o = (uint4 *)(dy + (size_t)v * 16);
                o[0] = make_uint4((uint32_t)to_bf16(scale * dh) | ((uint32_t)to_bf16(scale * dv) << 16), 0u, 0u, 0u);
                o[1] = make_uint4(0u, 0u, 0u, 0u);
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
// dbias[n] = sum_v dy[v][n] (slot 27, column 0). The contraction runs over
// voxels, so both MFMA operands must hold runs of voxels of one channel,
// while the activations and dy are channels-last. A block of 16 voxels x 16
// channels is made channel-major by v_mfma_f32_16x16x16bf16_1k against the
// identity (D = A I = A, exact in FP32, read out in the result layout: lane
// (c, kq) holds channel c of voxels 4kq .. 4kq+3), and two such blocks form
// the K = 32 operand of v_mfma_f32_16x16x32_bf16 (K slot 8kq + e is voxel
// 4kq + e of the first block for e < 4, of the second for e >= 4; dy and the
// input use the same order). The input slabs are staged by the convolution's
// frame walk; the shift of tap (dk, di, dj) is the staged position a block is
// read from, and one transposed block of staged row u serves the output rows
// u - di. A workgroup walks tiles of 16 output rows; each wavefront
// accumulates its share of the taps for four of those rows over all its
// items, the wavefronts then add their sums in LDS in a fixed order and the
// workgroup writes one partial [28][16][16] for the fixed-order reduction.
constexpr int kWgBlocks = 512;

struct WgradArgs {
    WalkGeom w;
    SlabSrc src;
    const uint16_t *dy;
    float *part;
};

// LDS transpose read (ds_read_b64_tr_b16): within each 16-lane group, lane i
// receives element e = 0..3 from component i & 3 of the 4 x 16-bit values that
// lane 4e + (i >> 2) points at.
typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s_t lds_v4s_t;
typedef __attribute__((address_space(3))) const uint2 lds_u2_t;

// Eight wavefronts: four row groups of the tile times two halves of the nine
// (dk, dj) offsets (5 and 4, the bias with the second half), so that each
// holds 15 tap accumulators and two wavefronts fit a SIMD.
constexpr int kWgNW = 8;

template <int CIN>
__global__ __launch_bounds__(64 * kWgNW, 2) void k_wgrad(const WgradArgs a)
{
    using St = SlabStage<CIN, kWgNW, 4>;
    using W = WalkShape<kWgNW, 4>;
    static_assert(28 * 256 * sizeof(float) <= W::RING * St::SLAB * sizeof(uint4), "the wavefront sums fit in the ring");
    __shared__ uint4 ring[W::RING * St::SLAB];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rg = wv & 3, th = wv >> 2; // row group, half of the (dk, dj) offsets
    const int row = lane & 15, kq = lane >> 4;
    const int te = row >> 2, tq = row & 3;
    const int nx = a.w.g.nx, ny = a.w.g.ny;

    // B operand of the transposing MFMA: the identity, B[4kq + e][n = row]
    bf16x4 ident;
#pragma unroll
    for (int e = 0; e < 4; ++e) ident[e] = 4 * kq + e == row ? (short)0x3f80 : (short)0;
    // B operand of the bias: ones in column 0
    bf16x8 ones0;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones0[e] = row == 0 ? (__bf16)1.0f : (__bf16)0.0f;

    // acc[ci][di]: tap (dk, di, dj) of the offset c = 5 th + ci = 3 dk + dj
    f32x4 acc[5][3], accb = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ci = 0; ci < 5; ++ci)
#pragma unroll
        for (int di = 0; di < 3; ++di) acc[ci][di] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // two transposed 16-voxel blocks as one K = 32 operand
    auto pair = [](f32x4 t0, f32x4 t1) {
        return __builtin_bit_cast(bf16x8, make_uint4(pack2_bf16(t0[0], t0[1]), pack2_bf16(t0[2], t0[3]),
                                                     pack2_bf16(t1[0], t1[1]), pack2_bf16(t1[2], t1[3])));
    };
    auto transpose = [&](uint2 x) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, x), ident,
                                                         f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
    };

    // dy of the row group's rows in frame k: lane (voxel row, kq) reads
    // channels 4kq .. 4kq+3; frame k + 1 is read while frame k is computed
    uint2 dyr[2][4][2];
    auto load_dy = [&](auto setc, int i0, int j0, int k) {
        constexpr int S = decltype(setc)::value;
        const int kc = min(k, a.w.g.B - 1); // past the last frame: read, never used
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const int i = i0 + kRowsPerWave * rg + r, j = j0 + 16 * sg + row;
                const size_t v = ((size_t)kc * nx + i) * ny + j;
                dyr[S][r][sg] = i < nx && j < ny ? *(const uint2 *)(a.dy + v * 16 + 4 * kq) : make_uint2(0u, 0u);
            }
    };

    St st;
    st.init(tid);
    frame_walk(a.w, a.src, ring, st, [&](auto setc, int s, int i0, int j0, int k, auto &&prefetch) {
        constexpr int S = decltype(setc)::value;
        prefetch();
        load_dy(std::integral_constant<int, 1 - S>{}, i0, j0, k + 1);
        if (i0 + kRowsPerWave * rg >= nx) return; // uniform per wavefront: no rows here
        bf16x8 ady[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ady[r] = pair(transpose(dyr[S][r][0]), transpose(dyr[S][r][1]));
            if (th == 1) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ady[r], ones0, accb, 0, 0, 0);
        }
#pragma unroll
        for (int ci = 0; ci < 5; ++ci) {
            const int c = 5 * th + ci;
            if (c >= 9) break; // uniform per wavefront
            const int dk = c / 3, dj = c % 3;
            const lds_u2_t *sl = (const lds_u2_t *)(ring + W::slot(s + dk) * St::SLAB);
#pragma unroll
            for (int u = 0; u < kRowsPerWave + 2; ++u) {
                // lane (row = 4 te + tq, kq) points the transposing read at
                // channels 4 tq .. 4 tq+3 of voxel 4 kq + te of block sg
                v4s_t tb[2];
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const int col = 16 * sg + 4 * kq + te + dj;
                    tb[sg] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                        (lds_v4s_t *)(sl + St::quarter_slot((kRowsPerWave * rg + u) * kSJ + col, col, tq)));
                }
                bf16x8 bx = __builtin_bit_cast(bf16x8, __builtin_shufflevector(tb[0], tb[1], 0, 1, 2, 3, 4, 5, 6, 7));
                // fp32 planes: channels 0-7 staged, quarters 2, 3 read 0, 1 again
                if (CIN == CIN_F32 && row >= 8) bx = bf16x8{};
#pragma unroll
                for (int di = 0; di < 3; ++di) {
                    const int r = u - di;
                    if (r < 0 || r >= kRowsPerWave) continue;
                    acc[ci][di] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ady[r], bx, acc[ci][di], 0, 0, 0);
                }
            }
        }
    }, [&](int i0, int j0, int k0) { load_dy(std::integral_constant<int, 0>{}, i0, j0, k0); });

    // acc: lane (c = row, kq) holds dW[t][4kq + e][c]. The row groups' sums
    // are added in LDS in a fixed order (row group 0 first).
    float *red = (float *)ring;
    for (int w = 0; w < kWgNW; ++w) {
        __syncthreads();
        if (wv == w) {
#pragma unroll
            for (int ci = 0; ci < 5; ++ci) {
                const int c = 5 * th + ci;
                if (c >= 9) break;
#pragma unroll
                for (int di = 0; di < 3; ++di)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int t = (c / 3) * 9 + di * 3 + c % 3;
                        const int idx = t * 256 + (4 * kq + e) * 16 + row;
                        red[idx] = rg == 0 ? acc[ci][di][e] : red[idx] + acc[ci][di][e];
                    }
            }
            if (th == 1)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int idx = 27 * 256 + (4 * kq + e) * 16 + row;
                    red[idx] = rg == 0 ? accb[e] : red[idx] + accb[e];
                }
        }
    }
    __syncthreads();
    float *p = a.part + (size_t)blockIdx.x * 28 * 256;
    for (int idx = tid; idx < 28 * 256; idx += 64 * kWgNW) p[idx] = red[idx];
}

// grad[t][n][c] = sum over groups in a fixed order: thread (entry, chunk)
// adds groups chunk, chunk + 8, ... of one of the block's 32 entries, and the
// eight chunk sums are added in order.
// (blockIdx.y: the layer, whose partials start kWgBlocks x 28 x 256 floats
// after the previous layer's)
__global__ __launch_bounds__(256) void k_wgrad_reduce(int ngroups, const float *__restrict__ part,
                                                      float *__restrict__ grad)
{
    __shared__ float lds[8][32];
    const int e = (int)threadIdx.x & 31, ch = (int)threadIdx.x >> 5;
    const int idx = blockIdx.x * 32 + e; // of 28 * 256 entries
    part += (size_t)blockIdx.y * kWgBlocks * 28 * 256;
    grad += (size_t)blockIdx.y * 28 * 256;
    float s = 0.0f;
    for (int b = ch; b < ngroups; b += 8) s += part[(size_t)b * 28 * 256 + idx];
    lds[ch][e] = s;
    __syncthreads();
    if (ch == 0) {
        float t = lds[0][e];
#pragma unroll
        for (int c = 1; c < 8; ++c) t += lds[c][e];
        grad[idx] = t;
    }
}

// Adam on the fp32 master parameters of the layers in the padded layout
// [28][16][16] (slot 27 column 0 = bias); entries outside a layer's real
// channels stay zero. Then repack bf16 weights for the forward (Wk[t][n][c])
// and transposed (WkT[t'][c][n], t' = mirrored tap) convolutions. blockIdx.y:
// the layer (input channels cin0 for the first, output channels coutL for the
// last, 16 otherwise); every array advances by one layer's size.
__global__ __launch_bounds__(256) void k_adam(int cin0, int coutL, float lr, float b1, float b2, float eps, float c1,
                                              float c2, const float *__restrict__ grad, float *__restrict__ w,
                                              float *__restrict__ m, float *__restrict__ v,
                                              uint16_t *__restrict__ Wk, uint16_t *__restrict__ WkT,
                                              float *__restrict__ bias)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= 28 * 256) return;
    const int l = blockIdx.y;
    const int cin = l == 0 ? cin0 : kNetHidden, cout = l == (int)gridDim.y - 1 ? coutL : kNetHidden;
    const size_t o = (size_t)l * 28 * 256;
    grad += o;
    w += o;
    m += o;
    v += o;
    Wk += (size_t)l * 27 * 256;
    WkT += (size_t)l * 27 * 256;
    bias += l * 16;
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

// Work split: tiles of ci x kCJ, each walked through runs of F frames; the
// frames are cut into runs only when there are fewer tiles than the
// resident workgroups (`slots`). Persistent grid of at most that many
// workgroups, each taking every gridDim-th item.
WalkGeom walk_geom(int nx, int ny, int B, int slots, int ci)
{
    WalkGeom w{};
    w.g = geom(nx, ny, B);
    const int nti = (nx + ci - 1) / ci;
    w.ntj = (ny + kCJ - 1) / kCJ;
    w.ntiles = nti * w.ntj;
    const int runs = std::max(1, std::min(B, (slots + w.ntiles - 1) / w.ntiles));
    w.F = (B + runs - 1) / runs;
    w.nitems = w.ntiles * ((B + w.F - 1) / w.F);
    return w;
}

template <int CIN, int COUT, bool RELU, bool GATE, bool PACK = false>
void launch_conv(ConvArgs a, int nx, int ny, int B, hipStream_t s)
{
    const int slots = conv_wgs_per_cu<CIN>() * device_cus();
    a.w = walk_geom(nx, ny, B, slots, WalkShape<kConvNW>::CI);
    hipLaunchKernelGGL((k_conv<CIN, COUT, RELU, GATE, PACK>), dim3(std::min(a.w.nitems, slots)), dim3(64 * kConvNW),
                       0, s, a);
}

ConvArgs conv_args(const uint16_t *Wk, const float *bias)
{
    ConvArgs a{};
    a.Wk = Wk;
    a.bias = bias;
    return a;
}

} // namespace

void wsnet_conv_input(int nx, int ny, int B, const float *x, const float *base, const uint16_t *Wk, const float *bias,
                      uint16_t *out16, uint8_t *sign, hipStream_t s)
{
    ConvArgs a = conv_args(Wk, bias);
    const size_t V = (size_t)nx * ny * B;
    a.src.x = x;
    a.src.xb0 = base ? base : x;
    a.src.xb1 = base ? base + V : x;
    a.src.xb_live = base != nullptr;
    a.out16 = out16;
    a.sign = sign;
    launch_conv<CIN_F32, COUT_BF16, true, false>(a, nx, ny, B, s);
}

void wsnet_conv(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, bool relu,
                const uint8_t *gate, uint16_t *out16, uint8_t *sign, hipStream_t s)
{
    ConvArgs a = conv_args(Wk, bias);
    a.src.in = in;
    a.gate = gate;
    a.out16 = out16;
    a.sign = sign;
    if (gate) launch_conv<CIN_BF16, COUT_BF16, false, true>(a, nx, ny, B, s);
    else if (relu) launch_conv<CIN_BF16, COUT_BF16, true, false>(a, nx, ny, B, s);
    else launch_conv<CIN_BF16, COUT_BF16, false, false>(a, nx, ny, B, s);
}

void wsnet_conv_out(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int cout,
                    float *y, hipStream_t s)
{
    ConvArgs a = conv_args(Wk, bias);
    a.src.in = in;
    a.out32 = y;
    a.cout = cout;
    if (cout <= 4) launch_conv<CIN_BF16, COUT_F32, false, false, true>(a, nx, ny, B, s);
    else launch_conv<CIN_BF16, COUT_F32, false, false>(a, nx, ny, B, s);
}

void wsnet_conv_dual(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int tv,
                     const float *base, float *dual, hipStream_t s)
{
    ConvArgs a = conv_args(Wk, bias);
    a.src.in = in;
    a.out32 = dual;
    a.obase = base;
    a.tv = tv;
    a.cout = 2;
    launch_conv<CIN_BF16, COUT_DUAL, false, false, true>(a, nx, ny, B, s);
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

int wsnet_wgrad(int nx, int ny, int B, const uint16_t *dy, const uint16_t *in, const float *x, const float *base,
                float *part, hipStream_t s)
{
    // one workgroup (two wavefronts per SIMD) per CU
    const int slots = std::min(device_cus(), kWgBlocks);
    WgradArgs a{};
    a.w = walk_geom(nx, ny, B, slots, WalkShape<kWgNW, 4>::CI);
    a.dy = dy;
    a.part = part;
    const int groups = std::min(a.w.nitems, slots);
    if (in) {
        a.src.in = in;
        hipLaunchKernelGGL(k_wgrad<CIN_BF16>, dim3(groups), dim3(64 * kWgNW), 0, s, a);
    } else {
        const size_t V = (size_t)nx * ny * B;
        a.src.x = x;
        a.src.xb0 = base ? base : x;
        a.src.xb1 = base ? base + V : x;
        a.src.xb_live = base != nullptr;
        hipLaunchKernelGGL(k_wgrad<CIN_F32>, dim3(groups), dim3(64 * kWgNW), 0, s, a);
    }
    return groups;
}

void wsnet_wgrad_reduce(int layers, int groups, const float *part, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(28 * 256 / 32, layers), dim3(256), 0, s, groups, part, grad);
}

void wsnet_adam(int layers, int cin0, int coutL, float lr, float b1, float b2, float eps, float c1, float c2,
                const float *grad, float *w, float *m, float *v, uint16_t *Wk, uint16_t *WkT, float *bias,
                hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(28, layers), dim3(256), 0, s, cin0, coutL, lr, b1, b2, eps, c1, c2, grad, w, m, v,
                       Wk, WkT, bias);
}

void wsnet_dual_from_net(int nx, int ny, int B, int tv, const float *y, const float *base, float *dual, hipStream_t s)
{
    const Geom g = geom(nx, ny, B);
    const uint32_t plane = (uint32_t)nx * ny;
    hipLaunchKernelGGL(k_dual_from_net, dim3((plane + 255) / 256), dim3(256), 0, s, g, tv, y, base, dual);
}

} // namespace sci
