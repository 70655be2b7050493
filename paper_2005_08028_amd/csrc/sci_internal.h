// Internal host-side declarations of libscitv: the context, its scratch
// buffers, and the kernel launchers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/scitv.h"

namespace sci {

// Growable device scratch buffer owned by a context.
struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

enum BufSlot {
    WS_DUAL0 = 0, WS_DUAL1, WS_DUAL2, WS_DUAL3, // rotating dual fields (p^(s-1), p^(s) in, two out)
    WS_THETA,                         // theta volume when the caller does not want it
    WS_SVOL,                          // ADMM denoiser input s = u + x
    WS_UVOL,                          // ADMM multiplier u
    WS_SINV,                          // 1 / (sum_k C_k^2 + rho) image
    WS_PARTIAL,                       // FP64 block partials of the reductions
    WS_XTMP,                          // denoiser input copy when X_in aliases the output
    WS_BATCH,                         // batched solve: per-problem Sinv and theta
    WS_BDESC,                         // batched solve: device problem table (eager path)
    WS_CBITS,                         // masks packed one bit per frame (+ a validity flag)
    WS_XNEXT,                         // TwIST: the third iterate buffer
    WS_VTVQ0, WS_VTVQ1,               // VTV: duals between the passes of one call as (p, p_prev) records
    WS_COUNT
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    void *owned = nullptr; // device memory the graph reads (freed with it)
};

void destroy_graph(GraphEntry &g);
// Destroy every captured graph (after a device synchronisation): the tiling
// they froze may no longer be the tuned one.
int drop_graphs(sci_ctx *ctx);

// Kernel families timed by the profiler.
enum ProfFamily { PF_FGP_STREAM = 0, PF_FGP_FUSED, PF_TV_THETA, PF_PROJECT, PF_SETUP, PF_COUNT };

struct ProfRec {
    int family;
    hipEvent_t a, b;
};

} // namespace sci

struct sci_ctx {
    int device = 0;
    int num_cus = 0;
    void *noalloc_scratch = nullptr; // device address of the fixed scratch array (sci_gap_tv_noalloc)
    std::string last_error;
    sci::Buf ws[sci::WS_COUNT];
    double *host_scalars = nullptr; // pinned, 8 doubles
    hipStream_t capture_stream = nullptr;
    std::map<std::string, sci::GraphEntry> graphs;
    // profiler: event pairs around launches (not recorded while capturing)
    bool prof_on = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<sci::ProfRec> prof;
    // fused-schedule tile shape chosen by the autotuner, per problem key
    std::map<std::string, std::pair<int, int>> tuned; // (tile shape, number of passes)
};

namespace sci {

// ---- fixed scratch of the allocation-free GAP entry point (noalloc.hip) -----
// Layout: 1 / S image (float per pixel), packed masks (32-bit word per
// pixel), the packed-mask flag; sized for nx * ny <= kNoAllocMaxPixels.
constexpr size_t kNoAllocMaxPixels = (size_t)1 << 22;
constexpr size_t kNoAllocBitsOffset = kNoAllocMaxPixels * 4;
constexpr size_t kNoAllocFlagOffset = kNoAllocBitsOffset + kNoAllocMaxPixels * 4;
constexpr size_t kNoAllocScratchBytes = kNoAllocFlagOffset + 256;
// Device address of the array on `device`, which must be current; looked up
// once per device and cached. SCI_OK or SCI_ERR_HIP.
int noalloc_scratch_lookup(int device, void **addr);

// ---- context helpers (ctx.cpp) ---------------------------------------------
int fail_hip(sci_ctx *ctx, hipError_t e, const char *what);
int fail(sci_ctx *ctx, int status, const std::string &msg);
int ensure_ws(sci_ctx *ctx, BufSlot slot, size_t bytes, hipStream_t stream);
int check_launch(sci_ctx *ctx, const char *what);
bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes);
size_t dual_elem_bytes(int dual_dtype);

// Scoped timing of the launches enqueued during its lifetime.
class ProfScope {
  public:
    ProfScope(sci_ctx *ctx, int family, hipStream_t s);
    ~ProfScope();

  private:
    sci_ctx *ctx_;
    int family_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
};

// ---- launchers (k_sensing.hip) ------------------------------------------------
void launch_forward(int nx, int ny, int B, const float *C, const float *X, float *Y, hipStream_t s);
void launch_adjoint(int nx, int ny, int B, const float *C, const float *Y, float *X, hipStream_t s);
void launch_weights(int nx, int ny, int B, const float *C, float rho, float *Sinv, hipStream_t s);
// x = theta + C .* ((Y - sum_k C_k theta_k) .* Sinv)
// GAP / ADMM projection. cbits / cflag (nullable): masks packed by
// launch_pack_masks; when *cflag is 1 the kernel reads the bits instead of C.
void launch_gap_project(int nx, int ny, int B, const float *theta, const float *C, const float *Y,
                        const float *Sinv, float *x, hipStream_t s, const uint32_t *cbits = nullptr,
                        const int *cflag = nullptr);
// v = theta - u; x = v + C .* ((Y - sum_k C_k v_k) .* Sinv); s = u + x
// (x nullable: then only s is stored)
void launch_admm_project(int nx, int ny, int B, const float *theta, const float *u, const float *C,
                         const float *Y, const float *Sinv, float *x, float *svol, hipStream_t s,
                         const uint32_t *cbits = nullptr, const int *cflag = nullptr);
// FISTA gradient step from the extrapolated point formed on load:
// v = x + ex (x - x_prev), z = v + C .* ((Y - sum_k C_k v_k) .* W)
void launch_fista_project(int nx, int ny, int B, const float *x, const float *x_prev, float ex, const float *C,
                          const float *Y, const float *W, float *z, hipStream_t s, const uint32_t *cbits = nullptr,
                          const int *cflag = nullptr);
// TwIST: the two-step update x_next = a0 x_prev + a1 x + a2 theta formed on
// load and stored (x_next must not overlap any input), then
// z = x_next + C .* ((Y - sum_k C_k x_next_k) .* W)
void launch_twist_project(int nx, int ny, int B, const float *x, const float *x_prev, const float *theta, float a0,
                          float a1, float a2, const float *C, const float *Y, const float *W, float *z, float *x_next,
                          hipStream_t s, const uint32_t *cbits = nullptr, const int *cflag = nullptr);
// bits[pix] bit k = (C_k(pix) == 1); *flag = 1 when every entry of C is 0 or 1
// and B <= 32, else 0 (all on the device: graph-capturable).
void launch_pack_masks(int nx, int ny, int B, const float *C, uint32_t *bits, int *flag, hipStream_t s);
void launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
void launch_fill(float *dst, float v, size_t n, hipStream_t s);
// theta = x + c (x - xp)
void launch_extrapolate(size_t n, float c, const float *x, const float *xp, float *th, hipStream_t s);
// out = a0 xp + a1 x + a2 th
void launch_two_step(size_t n, float a0, float a1, float a2, const float *xp, const float *x, const float *th,
                     float *out, hipStream_t s);
void launch_zero(void *dst, size_t bytes, hipStream_t s);

// ---- launchers (k_fgp.hip) ----------------------------------------------------
// One FGP iteration over HBM: p_next = P(w + D(x - lambda D^T w) / (8 lambda)),
// w = 0 (mode 0), w = p_cur (mode 1), w = p_cur + beta (p_cur - p_prev) (mode 2).
// VTV only (ATV and ITV2D stream through the tile kernel); other kinds
// return SCI_ERR_UNSUPPORTED.
int launch_fgp_stream(int tv, int dual_dtype, int nx, int ny, int B, const float *x, const void *p_cur,
                      const void *p_prev, void *p_next, int mode, float beta, float lam, hipStream_t s);
// The same iteration with Chambolle's (2004) semi-implicit step in place of
// the projection (every storage type and TV kind).
int launch_fgp_stream_chambolle04(int tv, int dual_dtype, int nx, int ny, int B, const float *x, const void *p_cur,
                                  const void *p_prev, void *p_next, int mode, float beta, float lam, hipStream_t s);
// One ATV-Clip iteration: w_next = per-direction clip(w + D theta_d / alpha,
// 2 lambda) with theta_d = x - D_d^T w_d; w nullable = zero (k_clip.hip).
// m (1..kTileMaxM) ATV-Clip iterations in one row-pipelined pass (k_clip_rows.hip):
// segments of H rows, starting duals w_in (nullable = zero), final duals to
// w_out (nullable), theta = x - D^T w and u = x - theta (nullable).
int launch_clip_rows(int H, int m, int nx, int ny, int B, const float *x, const float *w_in, float *w_out,
                     float alpha, float lambda, float *theta, float *u_out, hipStream_t s);
// One streaming ATV-Clip iteration, duals of any storage type.
int launch_clip(int dual_dtype, int nx, int ny, int B, const float *x, const void *w, void *w_next, float alpha,
                float lambda, hipStream_t s);
// theta = x - lambda D^T p; when u_out is non-null also u_out = x - theta.
int launch_tv_theta(int dual_dtype, int nx, int ny, int B, const float *x, const void *p, float lam,
                    float *theta, float *u_out, hipStream_t s);

// ---- launchers (k_fgp_tile.hip) -----------------------------------------------
// Fused schedule: m <= kTileMaxM inner iterations per pass over HBM.
constexpr int kTileMaxM = 10;
constexpr int kTuneSplits = 3; // pass counts tried by the autotuner: minimal, +1, +2
// b[0] forms w^(s0) from the loaded p^(s0), p^(s0-1) (mode 2); b[t+1] forms
// w^(s0+t+1) after iteration t of the pass.
struct TileBeta {
    float b[kTileMaxM + 1];
};
struct TilePass {
    const void *pc = nullptr;  // p^(s0) (mode 1, 2)
    const void *pp = nullptr;  // p^(s0-1) (mode 2)
    int mode = 0;              // 0: w = 0, 1: w = p^(s0), 2: w = p^(s0) + b[0] (p^(s0) - p^(s0-1))
    TileBeta beta{};
    void *pn_out = nullptr;    // p^(s0+m)      (nullable)
    void *pp_out = nullptr;    // p^(s0+m-1)    (nullable)
    float *theta = nullptr;    // x - lambda D^T p^(s0+m) (nullable)
    float *u_out = nullptr;    // x - theta     (nullable)
    // VTV projection passes: pc (quad_in) or pn_out (quad_out) is one record
    // (p_h, p_v, p_prev_h, p_prev_v) per voxel in the storage type instead of
    // the planar fields (pp / pp_out unused then); see vtv_rows_quad
    int quad_in = 0, quad_out = 0;
};
bool tile_supported(int tv);
int tile_shape_count();
bool tile_shape_info(int shape, int *rows, int *waves, int *cols);
// true for the row-pipelined shapes (numbered after the tiled ones)
bool tile_shape_pipelined(int shape);
// Row-pipelined VTV passes: the longest pass for B frames (0 when the kernel
// does not run them), and one pass of m iterations with the duals read and
// written between passes in dual_dtype (16-bit: projection step only).
int vtv_rows_max_pass(int B);
// The pass length the fused schedule splits a VTV call by when it is not told
// otherwise, with or without the dual records between passes: the kernel's
// longest, except where a shorter one measured faster (k_vtv_rows_kf1.hip).
int vtv_rows_auto_pass(int B, bool records);
// Whether a fused VTV pass of m iterations over B frames (projection step,
// any storage type) reads and writes the per-voxel dual records of TilePass.
bool vtv_rows_quad(int B, int m);
int launch_vtv_rows(int m, int nx, int ny, int B, const float *x, const TilePass &tp, float lam, hipStream_t s,
                    bool chambolle04 = false, int dual_dtype = 0);
// shape: index into the shape table (0 = default); 16-bit dual storage runs
// the default shape whatever is asked
// chambolle04: Chambolle's (2004) step instead of FGP (row-pipelined shapes,
// float32 duals, ATV and ITV2D)
int launch_fgp_tile(int tv, int dual_dtype, int m, int shape, int nx, int ny, int B, const float *x,
                    const TilePass &tp, float lam, hipStream_t s, bool chambolle04 = false);

// ---- launchers (k_reduce.hip) -------------------------------------------------
// Deterministic two-stage FP64 reductions into out_dev (device doubles).
int reduce_partial_blocks();
size_t gap_partial_doubles(int nx, int ny, int B, int tv);
// out_dev[0] = max_ij sum_k C_kij^2 (partials: reduce_partial_blocks() entries)
void launch_max_s(int nx, int ny, int B, const float *C, double *partials, double *out_dev, hipStream_t s);
void launch_sqdiff(int64_t n, const float *a, const float *b, double *partials, double *out_dev, hipStream_t s);
void launch_residual_sq(int nx, int ny, int B, const float *C, const float *X, const float *Y, double *partials,
                        double *out_dev, hipStream_t s);
// out_dev[0] = TV(theta), out_dev[1] = <D theta, p>, out_dev[2] = ||theta - x||^2;
// `partials` holds gap_partial_doubles(nx, ny, B, tv) doubles. VTV with
// B > 48: SCI_ERR_UNSUPPORTED, nothing launched.
int launch_gap_terms(int tv, int dual_dtype, int nx, int ny, int B, float lam, const float *x, const void *p,
                     double *partials, double *out_dev, hipStream_t s);

} // namespace sci
