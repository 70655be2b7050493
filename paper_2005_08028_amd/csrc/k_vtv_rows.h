// Row-pipelined fused-schedule denoiser for vectorial TV (ITV3D, Eq. (31)-(32)),
// instantiated in the k_vtv_rows_kf*.hip translation units.
//
// The temporal wavefront blocking of k_fgp_rows.h, for a TV whose projection
// couples all B frames of a pixel: a workgroup owns a strip of 64 columns
// (one per lane; a recomputed halo of M+1 columns on the left and M on the
// right) and a segment of H rows, and its ng wavefronts split the frames of
// every pixel, wavefront g holding frames [g*fpw, g*fpw + fpw) (KF >= fpw
// slots; a slot past the last frame reads frame B-1, stays out of the norm and
// stores nothing). All wavefronts walk the segment together, level t one row
// behind level t-1. At every level and step each wavefront forms q for its
// frames and their partial squared norm; the two steps of a 2-row chunk run
// one level apart, so that the partials of both travel in one exchange: they
// meet in LDS (one LDS-only barrier per round, double-buffered, all slots
// read in one fixed run) and are summed in wavefront order, so every
// wavefront scales its frames by the same per-pixel factor. Frame split
// and summation order are those of the streaming VTV pass, and the per-voxel
// arithmetic uses the same helpers in the same order: with float32 duals the
// results are bit-identical to streaming one iteration per pass.
//
// Each level reads x of its own row; x moves down the levels through
// registers (an LDS ring per frame would not fit next to B frames of state).
// Levels the pipeline fill has not reached are left out of the first chunks
// at compile time, as in the 2D kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "k_fgp_rows.h"
#include "sci_internal.h"
#include "sci_math.h"

namespace sci {

constexpr int kVtvMaxWaves = 8; // wavefronts (frame groups) per workgroup, at most

// MODE: 0 w = 0; 1 w = p^(s0); 2 w = p^(s0) + b[0] (p^(s0) - p^(s0-1)).
// CH_STEP = 1: Chambolle's (2004) semi-implicit step in place of the
// projection, |z/(8 lambda)| over all frames of the pixel, with the
// operations of the streaming pass. DT: storage type of the duals read and
// written between passes (arithmetic stays float32; 16-bit values are
// rounded to nearest even where they are stored).
// QIO: bit 0, p^(s0) and p^(s0-1) come as one record per voxel in pc; bit 1,
// p^(s0+m) and p^(s0+m-1) leave as one record in pn_out (projection step;
// the records of a call's intermediate passes, one load and one store instead
// of four; a 16-bit record holds the same rounded values as the four planar
// stores would).
// One voxel's dual record between passes: p_h, p_v, p_prev_h, p_prev_v in the
// storage type (8 or 16 bytes, moved by one load or store).
template <int DT> struct alignas(4 * sizeof(typename Dual<DT>::T)) DualRec {
    typename Dual<DT>::T v[4];
};

// Stores of this kernel in a 16-bit type: the hardware conversions (round to
// nearest even). For bfloat16 they give the bits of Dual<DT_BF16>::st on every
// non-NaN input, denormals included (checked over all 2^32 float patterns on
// the device), and a NaN stays a NaN; for binary16 they are Dual<DT_F16>::st.
typedef float vtv_f2 __attribute__((ext_vector_type(2)));
typedef __bf16 vtv_b2 __attribute__((ext_vector_type(2)));
typedef _Float16 vtv_h2 __attribute__((ext_vector_type(2)));

template <int DT> __device__ inline typename Dual<DT>::T vtv_to16(float v)
{
    if constexpr (DT == DT_BF16) return __builtin_bit_cast(uint16_t, (__bf16)v);
    else return (_Float16)v;
}

// two values packed into one word, the first in the low half
template <int DT> __device__ inline uint32_t vtv_pack16(float a, float b)
{
    const vtv_f2 f = {a, b};
    if constexpr (DT == DT_BF16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, vtv_b2));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, vtv_h2));
}

template <int M, int KF, int MODE, int CH_STEP, int DT = DT_F32, int QIO = 0>
__global__ __launch_bounds__(64 * kVtvMaxWaves) void k_vtv_rows(int nx, int ny, int B, int fpw, int nstrip, int H,
                                                              const float *__restrict__ x,
                                                              const typename Dual<DT>::T *__restrict__ pc,
                                                              const typename Dual<DT>::T *__restrict__ pp,
                                                              TileBeta bt, float lam, float step,
                                                              typename Dual<DT>::T *__restrict__ pn_out,
                                                              typename Dual<DT>::T *__restrict__ pp_out,
                                                              float *__restrict__ theta_out, float *__restrict__ u_out)
{
    using D = Dual<DT>;
    constexpr bool QIN = (QIO & 1) != 0, QOUT = (QIO & 2) != 0;
    static_assert(QIO == 0 || !CH_STEP, "dual records: projection passes");
    static_assert(!QIN || MODE >= 1, "a record input needs a dual start");
    constexpr int CH = kRowChunk;
    constexpr int TXO = 64 - 2 * M - 1; // interior columns per strip
    static_assert(TXO > 0, "strip too narrow for the pass length");
    static_assert(CH == 2, "steps run in pairs, one pair per chunk");
    __shared__ float2 n2s[2][kVtvMaxWaves][64]; // (step k, step k+1) partials

    const int ng = (int)(blockDim.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    const int lin = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int seg = lin / nstrip, sx = lin % nstrip;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t V = plane * (uint32_t)B;
    const int a = seg * H;         // first row of the segment
    const int hi = min(a + H, nx); // one past its last row
    const int j = sx * TXO - (M + 1) + lane;
    const bool jin = j >= 0 && j < ny;
    const bool hj = j >= 0 && j < ny - 1; // horizontal differences exist for 0 <= j < ny-1
    const float step_h = hj ? step : 0.0f;
    const uint32_t jcl = jin ? (uint32_t)j : 0u;
    const bool outc = lane >= M + 1 && lane <= 63 - M && j < ny;
    const int kbase = g * fpw;
    const int nk = max(0, min(fpw, B - kbase)); // real frames of this wavefront
    uint32_t fo[KF];
#pragma unroll
    for (int kk = 0; kk < KF; ++kk) fo[kk] = (uint32_t)min(kbase + kk, B - 1) * plane + jcl;

    // level t's state on its current row r, per frame slot
    float cth[M][KF], cwh[M][KF], cwv[M][KF], cph[M][KF], cpv[M][KF];
    // x of the rows the levels read: after the pair (k, k+1) starts, xl[t + 1]
    // is the row level t reads in step k and xl[t] the row it reads in step
    // k+1 (row k+2-t); xl[M+1] and xl[M] are the two theta rows
    float xl[M + 2][KF];
#pragma unroll
    for (int t = 0; t < M; ++t)
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) cth[t][kk] = cwh[t][kk] = cwv[t][kk] = cph[t][kk] = cpv[t][kk] = 0.0f;
#pragma unroll
    for (int t = 0; t <= M + 1; ++t)
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) xl[t][kk] = 0.0f;
    float cpm[KF]; // p_v^(s0+M) of the row above the theta row
#pragma unroll
    for (int kk = 0; kk < KF; ++kk) cpm[kk] = 0.0f;
    int par = 0; // LDS buffer of the next exchange
    // Every exchange reads all kVtvMaxWaves slots (one fixed run of LDS reads,
    // no loop over ng); the slots of absent wavefronts hold +0, which leaves
    // the non-negative sum unchanged. The first exchange's barrier orders
    // these writes before any read.
    for (int e = (int)threadIdx.x; e < 2 * kVtvMaxWaves * 64; e += (int)blockDim.x)
        if ((e >> 6) % kVtvMaxWaves >= ng) (&n2s[0][0][0])[e] = make_float2(0.0f, 0.0f);

    // Chunk loads of CH rows for every frame slot, from in-bounds addresses,
    // masked where consumed.
    float xn[CH][KF], lh[CH][KF], lv[CH][KF], mh[CH][KF], mv[CH][KF];
    auto load_chunk = [&](int i0) {
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int i = i0 + s;
            const uint32_t rowo = ((i >= 0 && i < nx) ? (uint32_t)i : 0u) * (uint32_t)ny;
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                const uint32_t o = fo[kk] + rowo;
                xn[s][kk] = x[o];
                if constexpr (QIN && DT == DT_F32) {
                    const float4 rec = ((const float4 *)pc)[o];
                    lh[s][kk] = rec.x;
                    lv[s][kk] = rec.y;
                    mh[s][kk] = rec.z;
                    mv[s][kk] = rec.w;
                } else if constexpr (QIN) {
                    const DualRec<DT> rec = ((const DualRec<DT> *)pc)[o];
                    lh[s][kk] = D::cvt(rec.v[0]);
                    lv[s][kk] = D::cvt(rec.v[1]);
                    mh[s][kk] = D::cvt(rec.v[2]);
                    mv[s][kk] = D::cvt(rec.v[3]);
                } else {
                    if (MODE >= 1) {
                        lh[s][kk] = D::ld(pc, o);
                        lv[s][kk] = D::ld(pc, V + o);
                    }
                    if (MODE == 2) {
                        mh[s][kk] = D::ld(pp, o);
                        mv[s][kk] = D::ld(pp, V + o);
                    }
                }
            }
        }
    };

    // Step k runs level t on row k - t (see k_fgp_rows.h for the timing).
    const int k_start = a - M - 2;
    const int nsteps = H + 2 * M + 1;
    const int nchunk = (nsteps + CH - 1) / CH; // >= M + 1 > NPRO
    constexpr int NPRO = (2 * (M - 1) + CH - 1) / CH;
    load_chunk(k_start + 1);
    auto chunk = [&](int b, auto pro) {
        constexpr int PB = decltype(pro)::value; // prologue chunk index, or -1
        const int k0 = k_start + b * CH;
        float i0h[CH][KF], i0v[CH][KF], j0h[CH][KF], j0v[CH][KF], x0[CH][KF];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int i = k0 + s + 1;
            const bool iin = i >= 0 && i < nx;
            const bool hin = iin && hj;                      // horizontal difference exists
            const bool vin = i >= 0 && i < nx - 1 && jin;    // vertical difference exists
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                x0[s][kk] = (iin && jin) ? xn[s][kk] : 0.0f;
                if (MODE == 0) {
                    i0h[s][kk] = i0v[s][kk] = j0h[s][kk] = j0v[s][kk] = 0.0f;
                } else {
                    j0h[s][kk] = hin ? lh[s][kk] : 0.0f;
                    j0v[s][kk] = vin ? lv[s][kk] : 0.0f;
                    if (MODE == 2) {
                        i0h[s][kk] = hin ? extrapolate(j0h[s][kk], mh[s][kk], bt.b[0]) : 0.0f;
                        i0v[s][kk] = vin ? extrapolate(j0v[s][kk], mv[s][kk], bt.b[0]) : 0.0f;
                    } else {
                        i0h[s][kk] = j0h[s][kk];
                        i0v[s][kk] = j0v[s][kk];
                    }
                }
            }
        }
        load_chunk(k0 + CH + 1);
        // The two steps of the chunk run skewed: in round tau, step k0 runs
        // level tau and step k0+1 level tau-1. (Step k, level t) needs only
        // (k, t-1) and (k-1, t), both finished in the round before, so the
        // two levels' partial norms share one exchange; each level's
        // arithmetic and each sum's order are those of one step at a time.
#pragma unroll
        for (int t = M + 1; t > 1; --t)
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) xl[t][kk] = xl[t - 2][kk];
#pragma unroll
        for (int kk = 0; kk < KF; ++kk) {
            xl[1][kk] = x0[0][kk];
            xl[0][kk] = x0[1][kk];
        }
        // a step's chain: w and p handed from level t to level t+1, and
        // p^(s0+M-1) of its output row
        float ih[2][KF], iv[2][KF], jh[2][KF], jv[2][KF], qph[2][KF], qpv[2][KF];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                ih[s][kk] = i0h[s][kk];
                iv[s][kk] = i0v[s][kk];
                jh[s][kk] = j0h[s][kk];
                jv[s][kk] = j0v[s][kk];
            }
#pragma unroll
        for (int tau = 0; tau <= M; ++tau) {
            // levels the pipeline fill has not reached stay idle (a level
            // idle in step k0+1 is idle in step k0 too)
            const bool runA = tau < M && !(PB >= 0 && PB * CH < 2 * tau);
            const bool runB = tau >= 1 && !(PB >= 0 && PB * CH + 1 < 2 * (tau - 1));
            if (!runA && !runB) break;
            float thn[2][KF], qh[2][KF], qv[2][KF], n2[2] = {0.0f, 0.0f};
            auto pre = [&](int sidx, int t) {
                const int r = k0 + sidx - t;
                const float step_v = (r >= 0 && r < nx - 1) ? step : 0.0f; // uniform per row
#pragma unroll
                for (int kk = 0; kk < KF; ++kk) {
                    thn[sidx][kk] = theta_of(xl[t + 1 - sidx][kk], from_left(ih[sidx][kk]), ih[sidx][kk], cwv[t][kk],
                                             iv[sidx][kk], lam);
                    const float zh = from_right(cth[t][kk]) - cth[t][kk];
                    const float zv = thn[sidx][kk] - cth[t][kk];
                    float n2a;
                    if (CH_STEP) {
                        const float sh = step_h * zh, sv = step_v * zv;
                        qh[sidx][kk] = cwh[t][kk] + sh;
                        qv[sidx][kk] = cwv[t][kk] + sv;
                        n2a = norm2_add(n2[sidx], sh, sv);
                    } else {
                        qh[sidx][kk] = ascend(cwh[t][kk], zh, step_h);
                        qv[sidx][kk] = ascend(cwv[t][kk], zv, step_v);
                        n2a = norm2_add(n2[sidx], qh[sidx][kk], qv[sidx][kk]);
                    }
                    n2[sidx] = kk < nk ? n2a : n2[sidx];
                }
            };
            auto post = [&](int sidx, int t, float tot) {
                const float sc = CH_STEP ? semi_implicit_scale(tot) : iso_scale(tot);
                const float bnext = bt.b[t + 1];
#pragma unroll
                for (int kk = 0; kk < KF; ++kk) {
                    const float nh = qh[sidx][kk] * sc, nv = qv[sidx][kk] * sc;
                    const float oh = extrapolate(nh, cph[t][kk], bnext);
                    const float ov = extrapolate(nv, cpv[t][kk], bnext);
                    if (t == M - 1) {
                        qph[sidx][kk] = cph[t][kk];
                        qpv[sidx][kk] = cpv[t][kk];
                    }
                    cth[t][kk] = thn[sidx][kk];
                    cwh[t][kk] = ih[sidx][kk];
                    cwv[t][kk] = iv[sidx][kk];
                    cph[t][kk] = jh[sidx][kk];
                    cpv[t][kk] = jv[sidx][kk];
                    ih[sidx][kk] = oh;
                    iv[sidx][kk] = ov;
                    jh[sidx][kk] = nh;
                    jv[sidx][kk] = nv;
                }
            };
            if (runA) pre(0, tau);
            if (runB) pre(1, tau - 1);
            n2s[par][g][lane] = make_float2(n2[0], n2[1]);
            lds_barrier();
            float totA = 0.0f, totB = 0.0f;
#pragma unroll
            for (int gg = 0; gg < kVtvMaxWaves; ++gg) {
                const float2 v2 = n2s[par][gg][lane];
                totA += v2.x;
                totB += v2.y;
            }
            par ^= 1;
            if (runA) post(0, tau, totA);
            if (runB) post(1, tau - 1, totB);
        }
        if (PB >= 0) return; // the theta rows are above the segment
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            // row r = k - M + 1 now has p^(s0+M) in jh, jv: theta = x - lambda D^T p
            const int r = k0 + s - M + 1;
            float th[KF];
#pragma unroll
            for (int kk = 0; kk < KF; ++kk) {
                th[kk] = theta_of(xl[M + 1 - s][kk], from_left(jh[s][kk]), jh[s][kk], cpm[kk], jv[s][kk], lam);
                cpm[kk] = jv[s][kk];
            }
            if (r >= a && r < hi && outc) {
                const uint32_t rowo = (uint32_t)r * (uint32_t)ny;
#pragma unroll
                for (int kk = 0; kk < KF; ++kk) {
                    if (kk >= nk) continue;
                    const uint32_t o = fo[kk] + rowo;
                    if (theta_out) theta_out[o] = th[kk];
                    if (u_out) u_out[o] = xl[M + 1 - s][kk] - th[kk];
                    if constexpr (QOUT && DT == DT_F32) {
                        ((float4 *)pn_out)[o] = make_float4(jh[s][kk], jv[s][kk], qph[s][kk], qpv[s][kk]);
                    } else if constexpr (QOUT) {
                        ((uint2 *)pn_out)[o] = make_uint2(vtv_pack16<DT>(jh[s][kk], jv[s][kk]),
                                                          vtv_pack16<DT>(qph[s][kk], qpv[s][kk]));
                    } else if constexpr (DT == DT_F32) {
                        if (pn_out) {
                            D::st(pn_out, o, jh[s][kk]);
                            D::st(pn_out, V + o, jv[s][kk]);
                        }
                        if (pp_out) {
                            D::st(pp_out, o, qph[s][kk]);
                            D::st(pp_out, V + o, qpv[s][kk]);
                        }
                    } else {
                        if (pn_out) {
                            pn_out[o] = vtv_to16<DT>(jh[s][kk]);
                            pn_out[V + o] = vtv_to16<DT>(jv[s][kk]);
                        }
                        if (pp_out) {
                            pp_out[o] = vtv_to16<DT>(qph[s][kk]);
                            pp_out[V + o] = vtv_to16<DT>(qpv[s][kk]);
                        }
                    }
                }
            }
        }
    };
    static_for<0, NPRO>([&](auto pb) { chunk(decltype(pb)::value, pb); });
    for (int b = NPRO; b < nchunk; ++b) chunk(b, std::integral_constant<int, -1>{});
}

} // namespace sci

namespace sci {

// Longest pass (inner iterations) the kernel runs without spilling
// registers, by frames per wavefront; 0 where it does not run.
constexpr int vtv_rows_max_m(int kf) { return kf == 1 ? 10 : kf == 2 ? 10 : kf == 3 ? 7 : kf == 4 ? 4 : 0; }

// Segment height. A step of the kernel is bound by the latency of its chain
// of norm exchanges, which a second workgroup on the same CU hides well and a
// third hardly (measured); so: up to two workgroups per CU, as registers
// allow, all in one round, and with that the tallest segments, which spend
// the least on the pipeline fill.
// Workgroups the launch aims at (CUs x co-resident workgroups, at most two),
// queried once per (kernel, workgroup size, device).
template <typename K>
long vtv_target_groups(K kernel, int ng)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, int>, long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_tuple((const void *)kernel, ng, dev);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int ncu = 0, nb = 0;
    if (dev < 0 || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 64 * ng, 0) != hipSuccess || nb < 1) nb = 1;
    const long target = (long)std::min(nb, 2) * ncu;
    cache.emplace(key, target);
    return target;
}

template <typename K>
int vtv_segment_rows(K kernel, int ng, int nx, int nstrip)
{
    const long target = vtv_target_groups(kernel, ng);
    const int nseg = (int)std::min<long>(std::max<long>(1, target / nstrip), std::max(1, nx));
    return (nx + nseg - 1) / nseg;
}

template <int M, int KF, int MODE, int CH_STEP, int DT, int QIO = 0>
void launch_vtv_mode(int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp, float lam,
                     hipStream_t s)
{
    using T = typename Dual<DT>::T;
    constexpr int TXO = 64 - 2 * M - 1;
    const int nstrip = (ny + TXO - 1) / TXO;
    const int H = vtv_segment_rows(k_vtv_rows<M, KF, MODE, CH_STEP, DT, QIO>, ng, nx, nstrip);
    const int nseg = (nx + H - 1) / H;
    hipLaunchKernelGGL((k_vtv_rows<M, KF, MODE, CH_STEP, DT, QIO>), dim3(nstrip * nseg), dim3(64 * ng), 0, s, nx, ny,
                       B, fpw, nstrip, H, x, (const T *)tp.pc, (const T *)tp.pp, tp.beta, lam, 1.0f / (8.0f * lam),
                       (T *)tp.pn_out, (T *)tp.pp_out, tp.theta, tp.u_out);
}

// Pass lengths with dual-record variants: projection passes of at least 3
// iterations at 2 to 4 frames per wavefront (multi-pass calls at one frame per
// wavefront need more than 10 iterations), at 2 frames up to 8; every storage
// type.
constexpr bool vtv_quad_inst(int kf, int m, int ch_step, int /*dt*/)
{
    return !ch_step && kf >= 2 && kf <= 4 && m >= 3 && m <= (kf == 2 ? 8 : vtv_rows_max_m(kf));
}

template <int M, int KF, int CH_STEP, int DT>
int launch_vtv_m(int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp, float lam,
                 hipStream_t s)
{
    const int qio = (tp.quad_in ? 1 : 0) | (tp.quad_out ? 2 : 0);
    if (qio == 0) {
        if (tp.mode == 0) launch_vtv_mode<M, KF, 0, CH_STEP, DT>(nx, ny, B, fpw, ng, x, tp, lam, s);
        else if (tp.mode == 1) launch_vtv_mode<M, KF, 1, CH_STEP, DT>(nx, ny, B, fpw, ng, x, tp, lam, s);
        else launch_vtv_mode<M, KF, 2, CH_STEP, DT>(nx, ny, B, fpw, ng, x, tp, lam, s);
        return SCI_OK;
    }
    if constexpr (vtv_quad_inst(KF, M, CH_STEP, DT)) {
        if (tp.mode == 0) {
            if (qio != 2) return SCI_ERR_INVALID_ARG; // a cold start reads no dual
            launch_vtv_mode<M, KF, 0, CH_STEP, DT, 2>(nx, ny, B, fpw, ng, x, tp, lam, s);
            return SCI_OK;
        }
#define SCI_VTV_Q(md)                                                                                                   if (qio == 1) launch_vtv_mode<M, KF, md, CH_STEP, DT, 1>(nx, ny, B, fpw, ng, x, tp, lam, s);                        else if (qio == 2) launch_vtv_mode<M, KF, md, CH_STEP, DT, 2>(nx, ny, B, fpw, ng, x, tp, lam, s);                   else launch_vtv_mode<M, KF, md, CH_STEP, DT, 3>(nx, ny, B, fpw, ng, x, tp, lam, s);
        if (tp.mode == 1) {
            SCI_VTV_Q(1)
        } else {
            SCI_VTV_Q(2)
        }
#undef SCI_VTV_Q
        return SCI_OK;
    }
    return SCI_ERR_UNSUPPORTED;
}

// Dispatch on the pass length m = 1..vtv_rows_max_m(KF).
template <int KF, int CH_STEP, int DT = DT_F32>
int launch_vtv_kf(int m, int nx, int ny, int B, int fpw, int ng, const float *x, const TilePass &tp, float lam,
                  hipStream_t s)
{
    constexpr int MM = vtv_rows_max_m(KF);
    if (m < 1 || m > MM) return SCI_ERR_INVALID_ARG;
    switch (m) {
#define SCI_VTV_M(mm)                                                                                               \
    case mm:                                                                                                        \
        if constexpr (mm <= MM) return launch_vtv_m<mm, KF, CH_STEP, DT>(nx, ny, B, fpw, ng, x, tp, lam, s);        \
        return SCI_OK;
        SCI_VTV_M(1) SCI_VTV_M(2) SCI_VTV_M(3) SCI_VTV_M(4) SCI_VTV_M(5) SCI_VTV_M(6) SCI_VTV_M(7) SCI_VTV_M(8)
        SCI_VTV_M(9) SCI_VTV_M(10)
#undef SCI_VTV_M
    }
    return SCI_ERR_INVALID_ARG;
}

} // namespace sci
