// Warm-start network kernels: a 4-layer 3x3x3 convolutional net over the
// (frame, row, column) volume that predicts the FGP dual field from the
// denoiser input, trained on (input, converged dual) pairs.
//
// Activations are channels-last bf16, [V][16] (V = B*nx*ny voxels, voxel
// v = (k*nx + i)*ny + j, 16 channels, unused channels zero). Weights are
// packed per layer as Wk[27][16 out][16 in] bf16 (tap t = (dk*3 + di)*3 + dj,
// offset (dk-1, di-1, dj-1)), with zero padding for the first layer's single
// input channel and the last layer's two output channels. Every convolution
// is an implicit GEMM on v_mfma_f32_16x16x16bf16_1k: a wavefront produces
// 16 voxels x 16 output channels, accumulating 27 MFMAs (one per tap, K = 16
// input channels) in FP32. Zero padding of the volume ("same" convolution)
// is a zero A operand for neighbours outside the volume.
//
// MFMA operand layout (checked on the hardware): lane l holds A row l%16 and
// B column l%16, with K elements 4*(l/16) .. 4*(l/16)+3; the result holds
// column l%16, rows 4*(l/16) .. 4*(l/16)+3.
#include <hip/hip_runtime.h>

#include "sci_internal.h"
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

// Linear index of the neighbour of voxel v at tap t (sign = +1 forward,
// -1 for the transposed convolution), or -1 outside the volume.
__device__ inline int64_t neighbour(const Geom &g, uint32_t v, int t, int sign)
{
    const int j = (int)(v % (uint32_t)g.ny);
    const uint32_t r = v / (uint32_t)g.ny;
    const int i = (int)(r % (uint32_t)g.nx);
    const int k = (int)(r / (uint32_t)g.nx);
    const int dk = t / 9 - 1, di = (t / 3) % 3 - 1, dj = t % 3 - 1;
    const int kk = k + sign * dk, ii = i + sign * di, jj = j + sign * dj;
    if (kk < 0 || kk >= g.B || ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) return -1;
    return ((int64_t)kk * g.nx + ii) * g.ny + jj;
}

constexpr int kConvWaves = 4;

// out[v][n] = sum_t sum_c Wk[t][n][c] in[nb(v, t)][c] (+ bias[n]); optional
// ReLU; optional mask by (gate[v][n] > 0) (ReLU derivative); output bf16
// [V][16] or, for the last layer, fp32 [V][16].
template <bool RELU, bool OUT_F32>
__global__ __launch_bounds__(64 * kConvWaves) void k_conv(Geom g, const uint16_t *__restrict__ in,
                                                          const uint16_t *__restrict__ Wk,
                                                          const float *__restrict__ bias, int sign,
                                                          const uint16_t *__restrict__ gate,
                                                          uint16_t *__restrict__ out16, float *__restrict__ out32)
{
    const int lane = threadIdx.x & 63;
    const uint32_t tile = blockIdx.x * kConvWaves + (threadIdx.x >> 6);
    const uint32_t v0 = tile * 16u;
    if (v0 >= g.V) return; // uniform per wavefront
    const int row = lane & 15, kq = lane >> 4;
    const uint32_t va = v0 + (uint32_t)row; // voxel of this lane's A row
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int t = 0; t < 27; ++t) {
        bf16x4 a = {0, 0, 0, 0};
        if (va < g.V) {
            const int64_t u = neighbour(g, va, t, sign);
            if (u >= 0) a = *(const bf16x4 *)(in + (size_t)u * 16 + kq * 4);
        }
        const bf16x4 b = *(const bf16x4 *)(Wk + ((size_t)t * 16 + row) * 16 + kq * 4);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    // result: column n = row (lane & 15), voxels v0 + 4*kq + e
    const int n = row;
    const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t v = v0 + 4u * kq + e;
        if (v >= g.V) continue;
        float y = acc[e] + bn;
        if (RELU) y = fmaxf(y, 0.0f);
        if (gate && !(from_bf16(gate[(size_t)v * 16 + n]) > 0.0f)) y = 0.0f;
        if (OUT_F32) out32[(size_t)v * 16 + n] = y;
        else out16[(size_t)v * 16 + n] = to_bf16(y);
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
                const double d = ((double)y[(size_t)v * 16 + c] + b) - (double)target[(size_t)c * V + v];
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

// Weight gradient: dW[t][n][c] = sum_v dy[v][n] in[nb(v, t)][c] and
// dbias[n] = sum_v dy[v][n], as MFMAs with the voxels as K. Each workgroup
// covers a fixed strided set of 16-voxel chunks and writes its partial sums
// (28 x 16 x 16 floats, slot 27 = bias in column 0) for a fixed-order second
// pass. Wavefront w of the group handles taps w, w+4, ...
constexpr int kWgradGroups = 512;
__global__ __launch_bounds__(256) void k_wgrad(Geom g, const uint16_t *__restrict__ dy,
                                               const uint16_t *__restrict__ in, float *__restrict__ part)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    constexpr int kTapsPerWave = 7; // 28 slots over 4 wavefronts
    f32x4 acc[kTapsPerWave];
#pragma unroll
    for (int q = 0; q < kTapsPerWave; ++q) acc[q] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    const uint32_t nchunk = (g.V + 15u) / 16u;
    for (uint32_t ch = blockIdx.x; ch < nchunk; ch += kWgradGroups) {
        // A[n][v'] = dy[v0 + v'][n]: lane holds n = row, v' = 4 kq + e
        bf16x4 a;
        uint32_t vv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            vv[e] = ch * 16u + 4u * kq + e;
            a[e] = vv[e] < g.V ? (short)dy[(size_t)vv[e] * 16 + row] : (short)0;
        }
#pragma unroll
        for (int q = 0; q < kTapsPerWave; ++q) {
            const int t = wv + 4 * q; // 0..27
            // B[v'][c] = in[nb(v0 + v', t)][c] (slot 27: 1 in column 0 for the bias)
            bf16x4 b;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                short val = 0;
                if (vv[e] < g.V) {
                    if (t == 27) {
                        val = row == 0 ? (short)0x3f80 : (short)0; // bf16 1.0
                    } else {
                        const int64_t u = neighbour(g, vv[e], t, 1);
                        if (u >= 0) val = (short)in[(size_t)u * 16 + row];
                    }
                }
                b[e] = val;
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
        }
    }
    // acc[q]: column c = row, rows n = 4 kq + e
    float *p = part + (size_t)blockIdx.x * 28 * 256;
#pragma unroll
    for (int q = 0; q < kTapsPerWave; ++q) {
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
            const float h = hin ? y[(size_t)v * 16] + (base ? base[v] : 0.0f) : 0.0f;
            const float w = vin ? y[(size_t)v * 16 + 1] + (base ? base[g.V + v] : 0.0f) : 0.0f;
            n2 = fmaf(w, w, fmaf(h, h, n2));
        }
    }
    const float svtv = fminf(1.0f, __builtin_amdgcn_rsqf(n2));
    for (int k = 0; k < g.B; ++k) {
        const uint32_t v = (uint32_t)k * plane + pix;
        float h = hin ? y[(size_t)v * 16] + (base ? base[v] : 0.0f) : 0.0f;
        float w = vin ? y[(size_t)v * 16 + 1] + (base ? base[g.V + v] : 0.0f) : 0.0f;
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

// The transposed convolution (data gradient) is this same convolution with
// the tap-mirrored, in/out-swapped weight pack WkT[26 - t][c][n] = W[t][n][c].
void wsnet_conv(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, bool relu,
                const uint16_t *gate, uint16_t *out16, float *out32, hipStream_t s)
{
    const Geom g = geom(nx, ny, B);
    const uint32_t tiles = (g.V + 15) / 16;
    const dim3 grid((tiles + kConvWaves - 1) / kConvWaves), block(64 * kConvWaves);
    const int sign = 1;
    if (out32) hipLaunchKernelGGL((k_conv<false, true>), grid, block, 0, s, g, in, Wk, bias, sign, gate, out16, out32);
    else if (relu) hipLaunchKernelGGL((k_conv<true, false>), grid, block, 0, s, g, in, Wk, bias, sign, gate, out16, out32);
    else hipLaunchKernelGGL((k_conv<false, false>), grid, block, 0, s, g, in, Wk, bias, sign, gate, out16, out32);
}

int wsnet_reduce_blocks() { return kRedBlocks; }
int wsnet_wgrad_groups() { return kWgradGroups; }

void wsnet_loss(int nx, int ny, int B, int cout, const float *y, const float *base, const float *target, uint16_t *dy,
                double *part, double *out, hipStream_t s)
{
    const uint32_t V = (uint32_t)nx * ny * B;
    hipLaunchKernelGGL(k_loss, dim3(kRedBlocks), dim3(256), 0, s, V, cout, y, base, target, dy, part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, s, kRedBlocks, (const double *)part, out);
}

void wsnet_wgrad(int nx, int ny, int B, const uint16_t *dy, const uint16_t *in, float *part, float *grad,
                 hipStream_t s)
{
    const Geom g = geom(nx, ny, B);
    hipLaunchKernelGGL(k_wgrad, dim3(kWgradGroups), dim3(256), 0, s, g, dy, in, part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(28), dim3(256), 0, s, kWgradGroups, (const float *)part, grad);
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
