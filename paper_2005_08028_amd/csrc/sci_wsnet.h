// Launchers of the warm-start network kernels (k_wsnet.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace sci {

constexpr int kNetLayers = 4;
constexpr int kNetHidden = 16;
constexpr int kNetSlots = 28 * 256; // per layer: [27 taps + bias][16 out][16 in] fp32 master layout

// 3x3x3 convolutions (Wk[27][16 out][16 in] bf16, bias nullable):
// sign bytes [V][4]: bit e of byte q set where channel 4q+e of a bf16 [V][16] field is > 0;
// first layer from fp32 planes x [V] and base [2][V] (nullable) with ReLU, to bf16 [V][16]
// (and its sign bytes, when sign is non-null);
void wsnet_conv_input(int nx, int ny, int B, const float *x, const float *base, const uint16_t *Wk, const float *bias,
                      uint16_t *out16, uint8_t *sign, hipStream_t s);
// bf16 [V][16] to bf16 [V][16], with ReLU, or zeroed where the gate's sign bit
// is clear (gate non-null, no ReLU); sign (nullable) as above;
void wsnet_conv(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, bool relu,
                const uint8_t *gate, uint16_t *out16, uint8_t *sign, hipStream_t s);
// bf16 [V][16] to the raw output planes y [cout][V] fp32;
void wsnet_conv_out(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int cout,
                    float *y, hipStream_t s);
// bf16 [V][16] to the dual [2][V] = (base +) output projected for tv 0 (ATV) or 1 (ITV2D).
void wsnet_conv_dual(int nx, int ny, int B, const uint16_t *in, const uint16_t *Wk, const float *bias, int tv,
                     const float *base, float *dual, hipStream_t s);
int wsnet_reduce_blocks();
int wsnet_wgrad_groups();
void wsnet_loss(int nx, int ny, int B, int cout, const float *y, const float *base, const float *target, uint16_t *dy,
                double *part, double *out, hipStream_t s);
// theta-space loss (1/V) sum (D^T (y + base - target))^2 over the two dual
// channels: g = D^T r into g [V], the bf16 gradient into dy, the sum of g^2
// into out[0] (part: wsnet_reduce_blocks() doubles).
int wsnet_loss_theta(int nx, int ny, int B, const float *y, const float *base, const float *target, float *g,
                     uint16_t *dy, double *part, double *out, hipStream_t s);
// weight-gradient partials of one layer into part (wsnet_wgrad_groups() x 28 x 256 floats): input bf16
// [V][16] `in`, or (in null) the first layer's fp32 planes x [V] and base [2][V] (nullable); returns the
// number of partials written
int wsnet_wgrad(int nx, int ny, int B, const uint16_t *dy, const uint16_t *in, const float *x, const float *base,
                float *part, hipStream_t s);
// sums `groups` partials of each of `layers` consecutive layer regions of part into grad [layers][28][256]
void wsnet_wgrad_reduce(int layers, int groups, const float *part, float *grad, hipStream_t s);
// Adam and the bf16 repack of `layers` consecutive layers (cin0: the first layer's input channels, coutL:
// the last layer's output channels)
void wsnet_adam(int layers, int cin0, int coutL, float lr, float b1, float b2, float eps, float c1, float c2,
                const float *grad, float *w, float *m, float *v, uint16_t *Wk, uint16_t *WkT, float *bias,
                hipStream_t s);
void wsnet_dual_from_net(int nx, int ny, int B, int tv, const float *y, const float *base, float *dual, hipStream_t s);

// input channels of a network (1: x; 3: x and a base dual)
int wsnet_input_channels(const sci_wsnet *n);

} // namespace sci
