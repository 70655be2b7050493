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
// input channels) in FP32. Blocks of the volume are staged in LDS with a
// zero-filled one-voxel halo, which is the zero padding of the "same"
// convolution.
//
// MFMA operand layout (checked on the hardware): lane l holds A row l%16 and
// B column l%16, with K elements 4*(l/16) .. 4*(l/16)+3; the result holds
// column l%16, rows 4*(l/16) .. 4*(l/16)+3.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// out[v][n] = sum_t sum_c Wk[t][n][c] in[nb(v, t)][c] (+ bias[n]); optional
// ReLU; optional mask by (gate[v][n] > 0) (ReLU derivative); output bf16
// [V][16] or, for the last layer, fp32 [V][16]. Computed over LDS tiles: a
// workgroup owns an output block of
// kTK frames x kTI rows x kTJ columns; it stages the block plus a one-voxel
// halo (all 16 channels, bf16, zero outside the volume) in LDS once, and its
// four wavefronts then run 16-voxel x 16-channel MFMA tiles along j, the A
// operand of each of the 27 taps read from LDS (8 bytes per lane) and the B
// operand (the weights of the tap) held in registers for the whole block.
// Two tiles are accumulated side by side to cover the MFMA latency.
constexpr int kTK = 4, kTI = 8, kTJ = 32;
constexpr int kHK = kTK + 2, kHI = kTI + 2, kHJ = kTJ + 2;
constexpr int kVoxStride = 18; // shorts per staged voxel (16 channels + 2 of padding: 36-byte stride, no bank conflicts)

template <bool RELU, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv_tile(Geom g, int ntj, int nti, const uint16_t *__restrict__ in,
                                                   const uint16_t *__restrict__ Wk, const float *__restrict__ bias,
                                                   const uint16_t *__restrict__ gate, uint16_t *__restrict__ out16,
                                                   float *__restrict__ out32)
{
    __shared__ uint16_t xs[kHK * kHI * kHJ * kVoxStride];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int bj = (int)blockIdx.x % ntj, bi = ((int)blockIdx.x / ntj) % nti, bk = (int)blockIdx.x / (ntj * nti);
    const int k0 = bk * kTK, i0 = bi * kTI, j0 = bj * kTJ;

    // stage the block and its halo: 8-byte chunks (4 channels), zero outside
    for (int e = threadIdx.x; e < kHK * kHI * kHJ * 4; e += 256) {
        const int q = e & 3, vox = e >> 2;
        const int jj = vox % kHJ, ii = (vox / kHJ) % kHI, kk = vox / (kHJ * kHI);
        const int k = k0 + kk - 1, i = i0 + ii - 1, j = j0 + jj - 1;
        bf16x4 v = {0, 0, 0, 0};
        if (k >= 0 && k < g.B && i >= 0 && i < g.nx && j >= 0 && j < g.ny)
            v = *(const bf16x4 *)(in + ((((size_t)k * g.nx + i) * g.ny + j) * 16 + q * 4));
        *(bf16x4 *)(xs + vox * kVoxStride + q * 4) = v;
    }
    // weights of every tap: B[k = input channel 4 kq + e][n = row]
    bf16x4 wb[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) wb[t] = *(const bf16x4 *)(Wk + ((size_t)t * 16 + row) * 16 + kq * 4);
    const float bn = bias ? bias[row] : 0.0f;
    __syncthreads();

    // output rows (kl, il) of the block: wavefront wv takes every fourth one;
    // each row holds kTJ / 16 = 2 MFMA tiles
    for (int rr = wv; rr < kTK * kTI; rr += 4) {
        const int kl = rr / kTI, il = rr % kTI;
        if (k0 + kl >= g.B || i0 + il >= g.nx) continue; // uniform per wavefront
        f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dk = t / 9, di = (t / 3) % 3, dj = t % 3; // offsets into the haloed block
            const int base = ((kl + dk) * kHI + (il + di)) * kHJ + dj + row;
            const bf16x4 a0 = *(const bf16x4 *)(xs + base * kVoxStride + kq * 4);
            const bf16x4 a1 = *(const bf16x4 *)(xs + (base + 16) * kVoxStride + kq * 4);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, wb[t], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, wb[t], acc1, 0, 0, 0);
        }
        // result of tile h: column n = row, voxels j = j0 + 16 h + 4 kq + e
        const size_t vrow = ((size_t)(k0 + kl) * g.nx + (i0 + il)) * g.ny;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = j0 + 16 * h + 4 * kq + e;
                if (j >= g.ny) continue;
                const size_t v = vrow + j;
                float y = (h == 0 ? acc0[e] : acc1[e]) + bn;
                if (RELU) y = fmaxf(y, 0.0f);
                if (gate && !(from_bf16(gate[v * 16 + row]) > 0.0f)) y = 0.0f;
                if (OUT_F32) out32[v * 16 + row] = y;
                else out16[v * 16 + row] = to_bf16(y);
            }
        }
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
    return (y[(size_t)v * 16] + b) - target[v];
}
__device__ inline float r_v(const float *y, const float *base, const float *target, uint32_t V, uint32_t v, bool ex)
{
    if (!ex) return 0.0f;
    const float b = base ? base[V + v] : 0.0f;
    return (y[(size_t)v * 16 + 1] + b) - target[V + v];
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
    const int ntj = (ny + kTJ - 1) / kTJ, nti = (nx + kTI - 1) / kTI, ntk = (B + kTK - 1) / kTK;
    const dim3 grid(ntj * nti * ntk), block(256);
    if (out32) hipLaunchKernelGGL((k_conv_tile<false, true>), grid, block, 0, s, g, ntj, nti, in, Wk, bias, gate, out16, out32);
    else if (relu) hipLaunchKernelGGL((k_conv_tile<true, false>), grid, block, 0, s, g, ntj, nti, in, Wk, bias, gate, out16, out32);
    else hipLaunchKernelGGL((k_conv_tile<false, false>), grid, block, 0, s, g, ntj, nti, in, Wk, bias, gate, out16, out32);
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
