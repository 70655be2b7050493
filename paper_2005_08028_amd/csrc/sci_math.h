// Per-voxel arithmetic of the TV denoiser (and the workgroup numbering),
// shared by every HIP kernel of the library so that the streaming and the
// fused schedules evaluate identical expressions (the build disables floating-point contraction; every fused
// multiply-add below is explicit).
//
// Notation follows Algorithm 1 (FGP box) of the paper: w is the extrapolated
// dual, theta = x - lambda D^T w, z = D theta, q = w + z / (8 lambda),
// p = projection of q onto the unit ball of the TV's dual norm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sci {

enum { TV_ATV = 0, TV_ITV2D = 1, TV_VTV = 2 };
enum { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2 };

// ---- dual storage types ---------------------------------------------------

template <int DT> struct Dual;

template <> struct Dual<DT_F32> {
    using T = float;
    __device__ static inline float cvt(T v) { return v; }
    __device__ static inline float ld(const T *p, uint32_t i) { return p[i]; }
    __device__ static inline void st(T *p, uint32_t i, float v) { p[i] = v; }
};

// bfloat16: upper half of a float32; stores round to nearest even.
template <> struct Dual<DT_BF16> {
    using T = uint16_t;
    __device__ static inline float cvt(T v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static inline float ld(const T *p, uint32_t i) { return cvt(p[i]); }
    __device__ static inline void st(T *p, uint32_t i, float v)
    {
        uint32_t u = __float_as_uint(v);
        uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
        if ((u & 0x7fffffffu) > 0x7f800000u) r = (u >> 16) | 0x40u; // keep NaN a NaN
        p[i] = (uint16_t)r;
    }
};

// IEEE binary16: hardware conversion (round to nearest even).
template <> struct Dual<DT_F16> {
    using T = _Float16;
    __device__ static inline float cvt(T v) { return (float)v; }
    __device__ static inline float ld(const T *p, uint32_t i) { return cvt(p[i]); }
    __device__ static inline void st(T *p, uint32_t i, float v) { p[i] = (_Float16)v; }
};

// ---- the FGP step ---------------------------------------------------------

// Extrapolated dual w = p + beta (p - p_prev).
__device__ inline float extrapolate(float p, float pp, float beta) { return fmaf(beta, p - pp, p); }

// theta = x - lambda (D^T w) with
// (D^T w)(i,j) = (w_h(i,j-1) - w_h(i,j)) + (w_v(i-1,j) - w_v(i,j));
// missing neighbours enter as 0.
__device__ inline float theta_of(float x, float wh_left, float wh, float wv_up, float wv, float lam)
{
    return fmaf(-lam, (wh_left - wh) + (wv_up - wv), x);
}

// q = w + step * z. Entries of the dual that carry no difference take
// step = 0 (so q = w, which is 0 there) instead of a masked z.
__device__ inline float ascend(float w, float z, float step) { return fmaf(step, z, w); }

// Cross-lane neighbours along j, as DPP wavefront shifts folded into the
// consuming instruction: the value held by lane l-1 (0 in lane 0), and by
// lane l+1 (0 in lane 63).
__device__ inline float from_left(float v) { return __builtin_amdgcn_update_dpp(0.0f, v, 0x138, 0xF, 0xF, true); }
__device__ inline float from_right(float v) { return __builtin_amdgcn_update_dpp(0.0f, v, 0x130, 0xF, 0xF, true); }

// ATV projection q / max(1, |q|): equal to clamping q to [-1, 1].
__device__ inline float proj_atv(float q) { return fminf(fmaxf(q, -1.0f), 1.0f); }

// Isotropic scale 1 / max(1, sqrt(n2)) = min(1, 1/sqrt(n2)) for a squared norm n2.
__device__ inline float iso_scale(float n2) { return fminf(1.0f, __builtin_amdgcn_rsqf(n2)); }

// Semi-implicit (Chambolle 2004) scale 1 / (1 + sqrt(n2)) for the squared
// norm n2 of z/(8 lambda), with the hardware square root and reciprocal
// (v_sqrt_f32, v_rcp_f32: about 1 ulp each, in place of the IEEE-exact
// sequences, which cost several times the instructions).
__device__ inline float semi_implicit_scale(float n2)
{
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_sqrtf(n2));
}

// The same step per component (ATV): q / (1 + |s|) for s = z/(8 lambda).
__device__ inline float semi_implicit_atv(float q, float s) { return q * __builtin_amdgcn_rcpf(1.0f + fabsf(s)); }

// Squared-norm accumulation (h^2 + v^2 added to acc).
__device__ inline float norm2_add(float acc, float h, float v) { return fmaf(v, v, fmaf(h, h, acc)); }

// ---- work mapping -----------------------------------------------------------

// Workgroups are handed to the 8 XCDs of the chip round-robin by linear id;
// renumber them so that XCD c gets one contiguous run of tiles (raster order
// within a frame), and tiles that share halos or cache lines share that
// XCD's L2.
__device__ inline int xcd_contiguous(int wg, int nwg)
{
    constexpr int kXcd = 8;
    const int q = nwg / kXcd, r = nwg % kXcd;
    const int c = wg % kXcd, idx = wg / kXcd;
    return c < r ? c * (q + 1) + idx : r * (q + 1) + (c - r) * q + idx;
}

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

} // namespace sci
