// Host drivers of libscitv: the TV denoiser loop (Algorithm 1, FGP / Cham
// boxes), GAP (Eq. (21)-(22)) and ADMM (Eq. (24)-(26)) outer loops, HIP-graph
// capture of the outer loop, and the FP64 metric entry points.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>

#include "k_fgp_tile_shapes.h"
#include "sci_internal.h"
#include "sci_wsnet.h"

namespace sci {
namespace {

inline size_t vol_elems(const sci_dims &d) { return (size_t)d.nx * d.ny * d.B; }
inline size_t img_elems(const sci_dims &d) { return (size_t)d.nx * d.ny; }

int use_device(sci_ctx *ctx)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipSetDevice");
    }
    return SCI_OK;
}

int check_dims(sci_ctx *ctx, const sci_dims &d)
{
    if (d.nx < 1 || d.ny < 1 || d.B < 1) return fail(ctx, SCI_ERR_INVALID_ARG, "nx, ny and B must be >= 1");
    if ((int64_t)d.nx * d.ny * d.B >= ((int64_t)1 << 31))
        return fail(ctx, SCI_ERR_INVALID_ARG, "B*nx*ny must be < 2^31");
    if (d.B > 65535) return fail(ctx, SCI_ERR_INVALID_ARG, "B must be <= 65535 (frames map to a grid dimension)");
    return SCI_OK;
}

int check_tv(sci_ctx *ctx, const sci_tv_params &p, const sci_dims &d)
{
    if (p.tv < SCI_TV_ATV || p.tv > SCI_TV_VTV) return fail(ctx, SCI_ERR_INVALID_ARG, "unknown tv kind");
    if (!std::isfinite(p.lambda) || p.lambda < 0.0f) return fail(ctx, SCI_ERR_INVALID_ARG, "lambda must be finite and >= 0");
    if (p.n_inner < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "n_inner must be >= 0");
    if (p.accel != 0 && p.accel != 1) return fail(ctx, SCI_ERR_INVALID_ARG, "accel must be 0 or 1");
    if (p.dual_dtype < SCI_DUAL_F32 || p.dual_dtype > SCI_DUAL_F16)
        return fail(ctx, SCI_ERR_INVALID_ARG, "unknown dual dtype");
    if (p.schedule < SCI_SCHED_AUTO || p.schedule > SCI_SCHED_FUSED)
        return fail(ctx, SCI_ERR_INVALID_ARG, "unknown schedule");
    if (p.tv == SCI_TV_VTV && d.B > 48)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "VTV denoiser supports B <= 48 frames");
    if (p.tv == SCI_TV_VTV && d.B > 32 && p.schedule == SCI_SCHED_FUSED)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "VTV with more than 32 frames runs on the streaming schedule only");
    if (p.tile_shape < 0 || p.tile_shape > tile_shape_count())
        return fail(ctx, SCI_ERR_INVALID_ARG, "tile_shape out of range");
    if (p.tile_passes < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "tile_passes must be >= 0");
    if (p.chambolle04 != 0 && p.chambolle04 != 1) return fail(ctx, SCI_ERR_INVALID_ARG, "chambolle04 must be 0 or 1");
    if (p.chambolle04 && p.dual_dtype != SCI_DUAL_F32 && p.schedule == SCI_SCHED_FUSED)
        return fail(ctx, SCI_ERR_UNSUPPORTED,
                    "the Chambolle-2004 step with 16-bit duals runs on the streaming schedule only");
    if (p.clip != 0 && p.clip != 1) return fail(ctx, SCI_ERR_INVALID_ARG, "clip must be 0 or 1");
    if (p.clip) {
        if (p.tv != SCI_TV_ATV) return fail(ctx, SCI_ERR_INVALID_ARG, "ATV-Clip is defined for anisotropic TV");
        if (!(p.clip_alpha >= 0.0f) || !std::isfinite(p.clip_alpha))
            return fail(ctx, SCI_ERR_INVALID_ARG, "clip_alpha must be finite and >= 0 (0 = 4)");
        if (p.chambolle04 || p.gap_tol > 0.0)
            return fail(ctx, SCI_ERR_UNSUPPORTED, "ATV-Clip runs a fixed iteration count");
        if (p.dual_dtype != SCI_DUAL_F32 && p.schedule == SCI_SCHED_FUSED)
            return fail(ctx, SCI_ERR_UNSUPPORTED, "ATV-Clip with 16-bit duals runs on the streaming schedule only");
    }
    return SCI_OK;
}

// FGP momentum nu^(s+1) = (1 + sqrt(1 + 4 nu^(s)^2)) / 2, nu^(0) = 1
// (Algorithm 1, FGP box); beta_s = (nu^(s) - 1) / nu^(s+1).
struct Momentum {
    double nu = 1.0;
    double step() // returns beta_s and advances s
    {
        const double nu1 = (1.0 + std::sqrt(1.0 + 4.0 * nu * nu)) / 2.0;
        const double b = (nu - 1.0) / nu1;
        nu = nu1;
        return b;
    }
};

// Relative duality gap gap / P(theta) of one check. A non-finite gap or
// primal (a NaN or infinity in the dual or the input) gives NaN, never a
// small number: primal > 0 is false for NaN, which must not read as 0.
double relative_gap(double gap, double primal)
{
    if (!std::isfinite(gap) || !std::isfinite(primal)) return std::numeric_limits<double>::quiet_NaN();
    return primal > 0.0 ? gap / primal : 0.0;
}

// Stopping test of the gap-controlled denoiser: NaN never meets a tolerance.
bool gap_met(double rel, double tol) { return std::isfinite(rel) && rel <= tol; }

// Dual-field bookkeeping of one denoiser call: four rotating scratch
// buffers, so that a pass never writes a buffer it (or another tile of it)
// reads: p^(s-1) and p^(s) in, up to two new fields out.
struct FgpRun {
    void *buf[4] = {nullptr, nullptr, nullptr, nullptr};
    void *quad[2] = {nullptr, nullptr}; // VTV: dual records between the passes of one call (when bound)
    size_t quad_bytes = 0;              // size of each record buffer
    const void *cur = nullptr;  // p^(s) (nullptr = zero)
    const void *prev = nullptr; // p^(s-1)
    int iters = 0;
    double beta_prev = 0.0; // beta_(s-1), used to form w^(s)
    Momentum mom;
    void *free_buffer(const void *also_exclude = nullptr) const
    {
        for (void *b : buf)
            if (b != cur && b != prev && b != also_exclude) return b;
        return nullptr;
    }
    int mode(const sci_tv_params &p) const
    {
        if (!cur) return 0;                                   // w = 0
        if (p.accel && iters > 0 && beta_prev != 0.0) return 2; // momentum
        return 1;                                             // w = p^(s)
    }
};

// Tile shape used for one-iteration passes when none is tuned (64 x 32 tiles, 8 wavefronts per
// SIMD: the fastest single-iteration shape measured at 1024x1024x24).
constexpr int kStreamTileShape = 3;

constexpr const char *kFusedScope =
    "the fused schedule covers ATV, ITV2D, and VTV with B <= 32 (the Chambolle-2004 step with float32 duals)";

int fgp_tile_iterate(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &p, const float *x, FgpRun &r, int n,
                     float *theta, float *u_out, bool keep_dual, hipStream_t s, int force_shape = -1,
                     int force_passes = -1);
int stream_tile_shape(const sci_ctx *ctx, const sci_tv_params &p, const sci_dims &d);

// Enqueue `n` more inner iterations of the streaming schedule: one pass over
// HBM per iteration. ATV and ITV2D run the tile kernel with one iteration per
// pass; VTV (all frames of a pixel coupled) runs the row-streaming kernel.
int fgp_iterate(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &p, const float *x, FgpRun &r, int n,
                hipStream_t s)
{
    if (tile_supported(p.tv) && !p.chambolle04)
        return fgp_tile_iterate(ctx, d, p, x, r, n, nullptr, nullptr, true, s, stream_tile_shape(ctx, p, d), n);
    for (int it = 0; it < n; ++it) {
        const int mode = r.mode(p);
        void *out = r.free_buffer();
        ProfScope prof(ctx, PF_FGP_STREAM, s);
        auto launch = p.chambolle04 ? launch_fgp_stream_chambolle04 : launch_fgp_stream;
        int st = launch(p.tv, p.dual_dtype, d.nx, d.ny, d.B, x, r.cur, r.prev ? r.prev : r.cur, out, mode,
                        (float)r.beta_prev, p.lambda, s);
        if (st != SCI_OK) return fail(ctx, st, "FGP pass not available for this request");
        st = check_launch(ctx, p.chambolle04 ? "Chambolle-2004 pass" : "k_fgp_groups");
        if (st != SCI_OK) return st;
        const double b = r.mom.step();
        r.beta_prev = p.accel ? b : 0.0;
        r.prev = r.cur;
        r.cur = out;
        ++r.iters;
    }
    return SCI_OK;
}

// Tuning key: the streaming schedule (one iteration per pass) is tuned
// separately from the multi-iteration passes.
std::string tune_key(const sci_tv_params &p, const sci_dims &d)
{
    char buf[128];
    snprintf(buf, sizeof buf, "%s|%d|%d|%d|%d|%d|%d", p.schedule == SCI_SCHED_STREAM ? "stream" : "fused", p.tv,
             p.dual_dtype, d.nx, d.ny, d.B, p.n_inner);
    return buf;
}

int stream_tile_shape(const sci_ctx *ctx, const sci_tv_params &p, const sci_dims &d)
{
    sci_tv_params q = p;
    q.schedule = SCI_SCHED_STREAM;
    auto it = ctx->tuned.find(tune_key(q, d));
    if (p.tile_shape >= 1) return p.tile_shape - 1;
    return it == ctx->tuned.end() ? kStreamTileShape : it->second.first;
}

constexpr int kDefaultPassLen = 5;

// Untuned choice among the row-pipelined shapes for passes of m iterations:
// each (frame, strip, segment) is one wavefront and about two run per SIMD,
// so a launch takes ceil(wavefronts / slots) rounds of (H + 2m + 1) row
// steps; the segment height with the fewest steps, provided its wavefronts
// fill at least half of the slots (smaller problems keep the 2D tile, whose
// workgroups hold many more wavefronts). -1 when no row shape qualifies.
int default_row_shape(const sci_ctx *ctx, const sci_dims &d, int m)
{
    const long slots = 2L * 4 * (ctx->num_cus > 0 ? ctx->num_cus : 256);
    const int txo = 64 * kRowCols - 2 * m - 1;
    const long nstrip = (d.ny + txo - 1) / txo;
    int best = -1;
    long best_cost = 0, best_waves = 0;
    for (int sh = 0; sh < tile_shape_count(); ++sh) {
        int H = 0, w = 0, c = 0;
        if (!tile_shape_pipelined(sh) || !tile_shape_info(sh, &H, &w, &c)) continue;
        const long waves = nstrip * ((d.nx + H - 1) / H) * d.B;
        const long cost = (waves + slots - 1) / slots * (H + 2L * m + 1);
        if (best < 0 || cost < best_cost) {
            best = sh;
            best_cost = cost;
            best_waves = waves;
        }
    }
    return best >= 0 && 2 * best_waves >= slots ? best : -1;
}

// Tile shape and number of passes of the fused schedule: explicit
// (tile_shape / tile_passes >= 1), else the autotuned choice for this
// problem, else, for a cold call of at most kTileMaxM iterations whose dual
// is not kept (one pass, no dual in or out, so any storage type: where the
// row-pipelined kernel measured faster than the tiles), a row-pipelined
// shape when the problem fills the chip, else shape 0 and passes of about
// kDefaultPassLen iterations.
void pick_tiling(const sci_ctx *ctx, const sci_tv_params &p, const sci_dims &d, int n, int *shape, int *npass,
                 bool single_cold_pass = false)
{
    *shape = 0;
    *npass = (n + kDefaultPassLen - 1) / kDefaultPassLen;
    auto it = ctx->tuned.find(tune_key(p, d));
    if (it != ctx->tuned.end()) {
        *shape = it->second.first;
        *npass = it->second.second;
    } else if (single_cold_pass && tile_supported(p.tv) && n >= 1 && n <= kTileMaxM) {
        const int rs = default_row_shape(ctx, d, n);
        if (rs >= 0) {
            *shape = rs;
            *npass = 1;
        }
    }
    if (p.tile_shape >= 1) *shape = p.tile_shape - 1;
    if (p.tile_passes >= 1) *npass = p.tile_passes;
    const int min_pass = (n + kTileMaxM - 1) / kTileMaxM;
    if (*npass < min_pass) *npass = min_pass;
    if (*npass > n) *npass = n;
}

int fgp_tile_iterate(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &p, const float *x, FgpRun &r, int n,
                     float *theta, float *u_out, bool keep_dual, hipStream_t s, int force_shape, int force_passes)
{
    int shape = 0, npass = 1;
    pick_tiling(ctx, p, d, n, &shape, &npass, !keep_dual && r.cur == nullptr);
    if (force_shape >= 0) shape = force_shape;
    if (force_passes >= 1) npass = force_passes;
    if (p.chambolle04 && p.tv != SCI_TV_VTV && !tile_shape_pipelined(shape)) { // only the row kernel has this step
        const int rs = default_row_shape(ctx, d, std::min(n, kTileMaxM));
        shape = rs >= 0 ? rs : kTileShapes + 1;
    }
    // VTV projection passes hand their duals to the next pass of the call as
    // one record per voxel in the storage type (one load and one store instead
    // of four), when every pass length of the split has that variant
    const bool records = p.tv == SCI_TV_VTV && !p.chambolle04 && r.quad[0] && r.quad[1] &&
                         r.quad_bytes >= 4 * vol_elems(d) * dual_elem_bytes(p.dual_dtype);
    if (p.tv == SCI_TV_VTV) { // untuned: the fewest passes of the automatic length, unless more are asked for
        const int mm = vtv_rows_auto_pass(d.B, records);
        if (mm < 1) return fail(ctx, SCI_ERR_UNSUPPORTED, kFusedScope);
        npass = std::min(n, std::max((n + mm - 1) / mm, p.tile_passes));
    }
    const bool quads = records && npass > 1 && vtv_rows_quad(d.B, n / npass) &&
                       vtv_rows_quad(d.B, n / npass + (n % npass ? 1 : 0));
    for (int q = 0; q < npass; ++q) {
        const int m = n / npass + (q < n % npass ? 1 : 0);
        const bool last = q == npass - 1;
        TilePass tp;
        tp.mode = r.mode(p);
        tp.pc = r.cur;
        tp.pp = r.prev ? r.prev : r.cur;
        tp.quad_in = quads && q > 0;
        tp.quad_out = quads && !last;
        tp.beta.b[0] = (float)r.beta_prev;
        double bl = r.beta_prev;
        for (int t = 0; t < m; ++t) {
            const double b = r.mom.step();
            bl = p.accel ? b : 0.0;
            tp.beta.b[t + 1] = (float)bl;
        }
        void *pn = tp.quad_out ? r.quad[q & 1] : (!last || keep_dual) ? r.free_buffer() : nullptr;
        // a one-iteration pass hands p^(s0) on as the next pass's p^(s-1);
        // without acceleration no pass extrapolates, and p^(s-1) is not kept
        void *ppn = (!tp.quad_out && (!last || keep_dual) && m > 1 && p.accel) ? r.free_buffer(pn) : nullptr;
        tp.pn_out = pn;
        tp.pp_out = ppn;
        tp.theta = last ? theta : nullptr;
        tp.u_out = last ? u_out : nullptr;
        ProfScope prof(ctx, m == 1 ? PF_FGP_STREAM : PF_FGP_FUSED, s);
        int st = launch_fgp_tile(p.tv, p.dual_dtype, m, shape, d.nx, d.ny, d.B, x, tp, p.lambda, s, p.chambolle04 != 0);
        if (st != SCI_OK) return fail(ctx, st, "fused FGP pass not available for this request");
        st = check_launch(ctx, "k_fgp_tile");
        if (st != SCI_OK) return st;
        r.beta_prev = bl;
        r.prev = tp.quad_out ? pn : (m == 1) ? r.cur : ppn; // a record holds both
        r.cur = pn;
        r.iters += m;
    }
    return SCI_OK;
}

// The four dual fields, and for fused VTV projection passes at 9 to 32 frames
// (2 to 4 frames per wavefront) the two record buffers of multi-pass calls
// (four values of the storage type per voxel).
int ensure_duals(sci_ctx *ctx, const sci_dims &d, int dual_dtype, hipStream_t s, const sci_tv_params *tv = nullptr)
{
    const size_t bytes = 2 * vol_elems(d) * dual_elem_bytes(dual_dtype);
    for (int k = 0; k < 4; ++k) {
        int st = ensure_ws(ctx, (BufSlot)(WS_DUAL0 + k), bytes, s);
        if (st != SCI_OK) return st;
    }
    if (tv && tv->tv == SCI_TV_VTV && !tv->chambolle04 && d.B > 8 && d.B <= 32)
        for (int k = 0; k < 2; ++k) {
            int st = ensure_ws(ctx, (BufSlot)(WS_VTVQ0 + k), 4 * vol_elems(d) * dual_elem_bytes(dual_dtype), s);
            if (st != SCI_OK) return st;
        }
    return SCI_OK;
}

// Binds the dual buffers; the record buffers with their size, which a pass
// checks against the records of its storage type and dims.
void bind_duals(sci_ctx *ctx, FgpRun &r)
{
    for (int k = 0; k < 4; ++k) r.buf[k] = ctx->ws[WS_DUAL0 + k].ptr;
    for (int k = 0; k < 2; ++k) r.quad[k] = ctx->ws[WS_VTVQ0 + k].ptr;
    r.quad_bytes = std::min(ctx->ws[WS_VTVQ0].bytes, ctx->ws[WS_VTVQ1].bytes);
}

// VTV on the fused schedule: the row-pipelined kernel (16-bit dual storage
// for the projection step, float32 for the Chambolle-2004 step).
bool vtv_fused_supported(const sci_tv_params &p, const sci_dims &d)
{
    return p.tv == SCI_TV_VTV && (p.dual_dtype == SCI_DUAL_F32 || !p.chambolle04) && !p.clip &&
           vtv_rows_max_pass(d.B) > 0;
}

bool fused_supported(const sci_tv_params &p, const sci_dims &d)
{
    if (p.clip) return p.tv == SCI_TV_ATV && p.dual_dtype == SCI_DUAL_F32; // row-pipelined clip kernel
    if (p.chambolle04) // row-pipelined kernels
        return p.dual_dtype == SCI_DUAL_F32 && (tile_supported(p.tv) || vtv_fused_supported(p, d));
    return tile_supported(p.tv) || vtv_fused_supported(p, d);
}

bool use_fused(const sci_tv_params &p, const sci_dims &d)
{
    if (p.schedule == SCI_SCHED_STREAM) return false;
    if (p.schedule == SCI_SCHED_FUSED) return true;
    return fused_supported(p, d) && p.n_inner >= 2;
}


// One denoiser call with a fixed iteration count, as used inside the outer
// loops: theta = x - lambda D^T p^(N), and u_out = x - theta when non-null.
// `warm` (nullable) holds the starting dual; when keep_dual is set the final
// dual is left in r.cur.
int denoise_fixed(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &p, const float *x, float *theta,
                  float *u_out, const void *warm, bool keep_dual, FgpRun &r, hipStream_t s)
{
    const size_t vb = vol_elems(d) * sizeof(float);
    r.cur = warm;
    r.prev = nullptr;
    r.iters = 0;
    r.beta_prev = 0.0;
    r.mom = Momentum();
    if (p.lambda == 0.0f || p.n_inner == 0) {
        launch_copy(x, theta, vb, s);
        if (u_out) launch_zero(u_out, vb, s);
        return check_launch(ctx, "copy");
    }
    if (p.clip) {
        // ATV-Clip: per-direction duals, output x - D^T w (lambda enters as the threshold)
        const float alpha = p.clip_alpha > 0.0f ? p.clip_alpha : 4.0f;
        if (use_fused(p, d)) { // row-pipelined passes of up to kTileMaxM iterations
            const int n = p.n_inner;
            int npass = std::max((n + kTileMaxM - 1) / kTileMaxM, p.tile_passes);
            npass = std::min(npass, n);
            int shape = p.tile_shape >= 1 ? p.tile_shape - 1 : -1;
            if (shape < 0 || !tile_shape_pipelined(shape)) {
                const int rs = default_row_shape(ctx, d, (n + npass - 1) / npass);
                shape = rs >= 0 ? rs : kTileShapes + 1;
            }
            int H = 0, w = 0, c = 0;
            tile_shape_info(shape, &H, &w, &c);
            for (int q = 0; q < npass; ++q) {
                const int m = n / npass + (q < n % npass ? 1 : 0);
                const bool last = q == npass - 1;
                float *out = (!last || keep_dual) ? (float *)r.free_buffer() : nullptr;
                ProfScope prof(ctx, PF_FGP_FUSED, s);
                int st = launch_clip_rows(H, m, d.nx, d.ny, d.B, x, (const float *)r.cur, out, alpha, p.lambda,
                                          last ? theta : nullptr, last ? u_out : nullptr, s);
                if (st != SCI_OK) return fail(ctx, st, "fused ATV-Clip pass");
                if ((st = check_launch(ctx, "k_clip_rows")) != SCI_OK) return st;
                r.prev = r.cur;
                r.cur = out;
                r.iters += m;
            }
            return SCI_OK;
        }
        for (int it = 0; it < p.n_inner; ++it) {
            void *out = r.free_buffer();
            ProfScope prof(ctx, PF_FGP_STREAM, s);
            int st = launch_clip(p.dual_dtype, d.nx, d.ny, d.B, x, r.cur, out, alpha, p.lambda, s);
            if (st != SCI_OK) return fail(ctx, st, "ATV-Clip pass");
            r.prev = r.cur;
            r.cur = out;
            ++r.iters;
        }
        int st = check_launch(ctx, "k_clip");
        if (st != SCI_OK) return st;
        ProfScope prof(ctx, PF_TV_THETA, s);
        st = launch_tv_theta(p.dual_dtype, d.nx, d.ny, d.B, x, r.cur, 1.0f, theta, u_out, s);
        if (st != SCI_OK) return fail(ctx, st, "theta pass");
        return check_launch(ctx, "k_tv_theta");
    }
    if (use_fused(p, d)) {
        if (!fused_supported(p, d)) return fail(ctx, SCI_ERR_UNSUPPORTED, kFusedScope);
        return fgp_tile_iterate(ctx, d, p, x, r, p.n_inner, theta, u_out, keep_dual, s);
    }
    if (tile_supported(p.tv) && !p.chambolle04)
        return fgp_tile_iterate(ctx, d, p, x, r, p.n_inner, theta, u_out, keep_dual, s, stream_tile_shape(ctx, p, d),
                                p.n_inner);
    int st = fgp_iterate(ctx, d, p, x, r, p.n_inner, s);
    if (st != SCI_OK) return st;
    ProfScope prof(ctx, PF_TV_THETA, s);
    st = launch_tv_theta(p.dual_dtype, d.nx, d.ny, d.B, x, r.cur, p.lambda, theta, u_out, s);
    if (st != SCI_OK) return fail(ctx, st, "theta pass");
    return check_launch(ctx, "k_tv_theta");
}

// Relative duality gap lambda (TV - <D theta, p>) / P(theta) of the dual p,
// computed in FP64 on the GPU and read back (synchronises the stream).
int rel_gap(sci_ctx *ctx, const sci_dims &d, int tv, int dual_dtype, float lam, const float *x, const void *p,
            double *gap, double *primal, hipStream_t s)
{
    const size_t np = gap_partial_doubles(d.nx, d.ny, d.B, tv);
    int st = ensure_ws(ctx, WS_PARTIAL, (np + 8) * sizeof(double), s);
    if (st != SCI_OK) return st;
    double *part = (double *)ctx->ws[WS_PARTIAL].ptr;
    double *outd = part + np;
    if (!p) {
        st = ensure_ws(ctx, WS_DUAL2, 2 * vol_elems(d) * dual_elem_bytes(dual_dtype), s);
        if (st != SCI_OK) return st;
        launch_zero(ctx->ws[WS_DUAL2].ptr, 2 * vol_elems(d) * dual_elem_bytes(dual_dtype), s);
        p = ctx->ws[WS_DUAL2].ptr;
    }
    st = launch_gap_terms(tv, dual_dtype, d.nx, d.ny, d.B, lam, x, p, part, outd, s);
    if (st != SCI_OK) return fail(ctx, st, "duality gap: VTV supports B <= 48 frames");
    st = check_launch(ctx, "k_gap_rows");
    if (st != SCI_OK) return st;
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, outd, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
    const double tvv = ctx->host_scalars[0], inner = ctx->host_scalars[1], fid = ctx->host_scalars[2];
    *gap = (double)lam * (tvv - inner);
    *primal = 0.5 * fid + (double)lam * tvv;
    return SCI_OK;
}

// ---- outer loops ---------------------------------------------------------------

// Scratch for the packed masks: one 32-bit word per pixel, then the flag.
size_t cbits_bytes(const sci_dims &d) { return ((img_elems(d) * sizeof(uint32_t) + 255) & ~(size_t)255) + 256; }
uint32_t *cbits_ptr(sci_ctx *ctx) { return (uint32_t *)ctx->ws[WS_CBITS].ptr; }
int *cflag_ptr(sci_ctx *ctx, const sci_dims &d)
{
    return (int *)((char *)ctx->ws[WS_CBITS].ptr + ((img_elems(d) * sizeof(uint32_t) + 255) & ~(size_t)255));
}

// One outer solve: its inputs, outputs and the device scratch it runs on
// (the context's growable buffers, or the fixed array of the allocation-free
// entry point).
struct OuterArgs {
    sci_dims d;
    sci_solver_params p;
    const float *Y, *C, *X_init;
    float *X_out, *theta;
    bool admm;
    float *Sinv;               // 1 / (S + rho) image
    uint32_t *cbits;           // packed masks, one word per pixel
    int *cflag;                // 1 when the packed masks apply
    float *svol, *u;           // ADMM only
    void *duals[4];            // dual fields (nullptr: none needed)
    void *quads[2];            // VTV dual records between passes (nullptr: not used)
    size_t quad_bytes;         // size of each record buffer
};

int enqueue_outer(sci_ctx *ctx, const OuterArgs &a, hipStream_t s)
{
    const sci_dims &d = a.d;
    const size_t vb = vol_elems(d) * sizeof(float);
    float *Sinv = a.Sinv;
    float *theta = a.theta;
    float *svol = a.admm ? a.svol : nullptr;
    float *u = a.admm ? a.u : nullptr;
    uint32_t *cbits = a.cbits;
    int *cflag = a.cflag;

    {
        ProfScope prof(ctx, PF_SETUP, s);
        launch_weights(d.nx, d.ny, d.B, a.C, a.admm ? a.p.rho : 0.0f, Sinv, s);
        launch_pack_masks(d.nx, d.ny, d.B, a.C, cbits, cflag, s);
        if (a.X_init) launch_copy(a.X_init, theta, vb, s);     // theta^(0) = X_init
        else launch_adjoint(d.nx, d.ny, d.B, a.C, a.Y, theta, s); // theta^(0) = Phi^T y
        if (a.admm) launch_zero(u, vb, s);                     // u^(0) = 0
    }
    int st = check_launch(ctx, "outer setup");
    if (st != SCI_OK) return st;
    if (a.p.outer_iters == 0) {
        launch_copy(theta, a.X_out, vb, s);
        return check_launch(ctx, "copy");
    }
    FgpRun r;
    for (int k = 0; k < 4; ++k) r.buf[k] = a.duals[k];
    r.quad[0] = a.quads[0];
    r.quad[1] = a.quads[1];
    r.quad_bytes = a.quad_bytes;
    const void *warm = nullptr;
    for (int t = 0; t < a.p.outer_iters; ++t) {
        if (!a.admm) {
            {
                ProfScope prof(ctx, PF_PROJECT, s);
                launch_gap_project(d.nx, d.ny, d.B, theta, a.C, a.Y, Sinv, a.X_out, s, cbits, cflag);
            }
            st = check_launch(ctx, "k_project");
            if (st != SCI_OK) return st;
            st = denoise_fixed(ctx, d, a.p.tv, a.X_out, theta, nullptr, warm, a.p.warm_dual != 0, r, s);
        } else {
            {
                // x^(t) feeds only the output: the denoiser reads s = u + x and
                // forms u = s - theta itself, so x is stored on the last pass only
                float *x = t + 1 == a.p.outer_iters ? a.X_out : nullptr;
                ProfScope prof(ctx, PF_PROJECT, s);
                launch_admm_project(d.nx, d.ny, d.B, theta, u, a.C, a.Y, Sinv, x, svol, s, cbits, cflag);
            }
            st = check_launch(ctx, "k_project");
            if (st != SCI_OK) return st;
            // theta = TVdenoise(s); u = s - theta  (= u + x - theta)
            st = denoise_fixed(ctx, d, a.p.tv, svol, theta, u, warm, a.p.warm_dual != 0, r, s);
        }
        if (st != SCI_OK) return st;
        if (a.p.warm_dual) warm = r.cur;
    }
    return SCI_OK;
}

std::string graph_key(const OuterArgs &a)
{
    char buf[512];
    const sci_tv_params &t = a.p.tv;
    snprintf(buf, sizeof buf, "%d|%d,%d,%d|%d,%.9g,%d,%d,%d,%d,%d,%d,%d,%d,%.9g|%d,%.9g,%d|%p,%p,%p,%p,%p",
             a.admm ? 1 : 0, a.d.nx, a.d.ny, a.d.B, t.tv, (double)t.lambda, t.n_inner, t.accel, t.dual_dtype,
             t.schedule, t.chambolle04, t.tile_shape, t.tile_passes, t.clip, (double)t.clip_alpha, a.p.outer_iters,
             (double)a.p.rho, a.p.warm_dual, (const void *)a.Y, (const void *)a.C, (const void *)a.X_init,
             (void *)a.X_out, (void *)a.theta);
    return buf;
}

// Argument checks shared by the outer-loop entry points.
int check_outer_args(sci_ctx *ctx, const sci_dims &d, const sci_solver_params *p, const float *Y, const float *C,
                     float *X_out, float *Theta_out, const float *X_init)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!p || !Y || !C || !X_out) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    st = check_tv(ctx, p->tv, d);
    if (st != SCI_OK) return st;
    if (p->outer_iters < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "outer_iters must be >= 0");
    if (!std::isfinite(p->rho) || p->rho < 0.0f) return fail(ctx, SCI_ERR_INVALID_ARG, "rho must be finite and >= 0");
    if (p->warm_dual != 0 && p->warm_dual != 1) return fail(ctx, SCI_ERR_INVALID_ARG, "warm_dual must be 0 or 1");
    const size_t vb = vol_elems(d) * sizeof(float), ib = img_elems(d) * sizeof(float);
    const void *ins[3] = {Y, C, X_init};
    const size_t inb[3] = {ib, vb, vb};
    for (int k = 0; k < 3; ++k)
        if (overlaps(X_out, vb, ins[k], inb[k]) || overlaps(Theta_out, vb, ins[k], inb[k]))
            return fail(ctx, SCI_ERR_ALIAS, "outputs must not overlap Y, C or X_init");
    if (overlaps(X_out, vb, Theta_out, vb)) return fail(ctx, SCI_ERR_ALIAS, "X_out and Theta_out overlap");
    return use_device(ctx);
}

int run_outer(sci_ctx *ctx, const sci_dims &d, const sci_solver_params *p, const float *Y, const float *C,
              float *X_out, float *Theta_out, const float *X_init, bool admm, hipStream_t s)
{
    int st = check_outer_args(ctx, d, p, Y, C, X_out, Theta_out, X_init);
    if (st != SCI_OK) return st;
    const size_t vb = vol_elems(d) * sizeof(float), ib = img_elems(d) * sizeof(float);

    // scratch first: a graph must never see a buffer that later grows
    if ((st = ensure_ws(ctx, WS_SINV, ib, s)) != SCI_OK) return st;
    if (!Theta_out && (st = ensure_ws(ctx, WS_THETA, vb, s)) != SCI_OK) return st;
    if (admm && ((st = ensure_ws(ctx, WS_SVOL, vb, s)) != SCI_OK || (st = ensure_ws(ctx, WS_UVOL, vb, s)) != SCI_OK))
        return st;
    if ((st = ensure_duals(ctx, d, p->tv.dual_dtype, s, &p->tv)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_CBITS, cbits_bytes(d), s)) != SCI_OK) return st;

    OuterArgs a{d, *p, Y, C, X_init, X_out, Theta_out ? Theta_out : (float *)ctx->ws[WS_THETA].ptr, admm,
                (float *)ctx->ws[WS_SINV].ptr, cbits_ptr(ctx), cflag_ptr(ctx, d),
                admm ? (float *)ctx->ws[WS_SVOL].ptr : nullptr, admm ? (float *)ctx->ws[WS_UVOL].ptr : nullptr,
                {nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr}, 0};
    for (int k = 0; k < 4; ++k) a.duals[k] = ctx->ws[WS_DUAL0 + k].ptr;
    {
        FgpRun rb;
        bind_duals(ctx, rb);
        a.quads[0] = rb.quad[0];
        a.quads[1] = rb.quad[1];
        a.quad_bytes = rb.quad_bytes;
    }
    if (!p->use_graph) return enqueue_outer(ctx, a, s);

    const std::string key = graph_key(a);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamBeginCapture");
        ctx->capturing = true;
        st = enqueue_outer(ctx, a, ctx->capture_stream);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->capture_stream, &g);
        if (st != SCI_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipGraphInstantiate");
        it = ctx->graphs.emplace(key, GraphEntry{exec, nullptr}).first;
    }
    hipError_t e = hipGraphLaunch(it->second.exec, s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipGraphLaunch");
    return SCI_OK;
}

int read_scalars(sci_ctx *ctx, const double *dev, int n, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, dev, n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
    return SCI_OK;
}

// L(f) = max_ij S_ij, the largest eigenvalue of Phi^T Phi (read back; synchronises).
int lipschitz(sci_ctx *ctx, const sci_dims &d, const float *C, double *L, hipStream_t s)
{
    const int nb = reduce_partial_blocks();
    int st = ensure_ws(ctx, WS_PARTIAL, (3 * (size_t)nb + 8) * sizeof(double), s);
    if (st != SCI_OK) return st;
    double *part = (double *)ctx->ws[WS_PARTIAL].ptr;
    double *outd = part + 3 * nb;
    launch_max_s(d.nx, d.ny, d.B, C, part, outd, s);
    if ((st = check_launch(ctx, "k_max_s")) != SCI_OK) return st;
    if ((st = read_scalars(ctx, outd, 1, s)) != SCI_OK) return st;
    *L = ctx->host_scalars[0];
    return SCI_OK;
}

// TwIST's alpha, beta for the spectrum bounds [xi1, 1] of Phi^T Phi / L:
// rho = (1 - sqrt(xi1)) / (1 + sqrt(xi1)), alpha = 1 + rho^2, beta = 2 alpha / (xi1 + 1).
constexpr double kTwistXi1 = 0.1;
void twist_defaults(double *alpha, double *beta)
{
    const double k = std::sqrt(kTwistXi1);
    const double rho = (1.0 - k) / (1.0 + k);
    *alpha = 1.0 + rho * rho;
    *beta = 2.0 * *alpha / (kTwistXi1 + 1.0);
}

// FISTA and TwIST (Sec. 2.2) on 1/2 ||y - Phi x||^2 + lambda TV(x): gradient
// step z = v + (1/L) Phi^T (y - Phi v) (the GAP projection kernel with the
// constant weight 1/L), denoiser with weight lambda / L, then the FISTA
// extrapolation or the TwIST two-step update. Eager only: L is read back.
int run_prox_grad(sci_ctx *ctx, const sci_dims &d, const sci_solver_params *p, const float *Y, const float *C,
                  float *X_out, float *Theta_out, const float *X_init, bool twist, hipStream_t s)
{
    int st = check_outer_args(ctx, d, p, Y, C, X_out, Theta_out, X_init);
    if (st != SCI_OK) return st;
    if (p->use_graph) return fail(ctx, SCI_ERR_UNSUPPORTED, "FISTA / TwIST run eagerly (L(f) is read back)");
    double alpha = p->twist_alpha, beta = p->twist_beta;
    if (twist) {
        if (alpha == 0.0 && beta == 0.0) twist_defaults(&alpha, &beta);
        if (!(alpha > 0.0 && alpha < 2.0) || !(beta > 0.0) || !std::isfinite(beta))
            return fail(ctx, SCI_ERR_INVALID_ARG, "TwIST needs 0 < alpha < 2 and beta > 0 (or both 0 for defaults)");
    }
    const size_t V = vol_elems(d), vb = V * sizeof(float), ib = img_elems(d) * sizeof(float);
    if ((st = ensure_ws(ctx, WS_SINV, ib, s)) != SCI_OK) return st;
    if (!Theta_out && (st = ensure_ws(ctx, WS_THETA, vb, s)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_SVOL, vb, s)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_XTMP, vb, s)) != SCI_OK) return st;
    if (twist && (st = ensure_ws(ctx, WS_XNEXT, vb, s)) != SCI_OK) return st;
    if ((st = ensure_duals(ctx, d, p->tv.dual_dtype, s, &p->tv)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_CBITS, cbits_bytes(d), s)) != SCI_OK) return st;
    double L = 0.0;
    if ((st = lipschitz(ctx, d, C, &L, s)) != SCI_OK) return st;
    if (!(L > 0.0)) return fail(ctx, SCI_ERR_INVALID_ARG, "every mask entry is zero (L(f) = 0)");
    float *W = (float *)ctx->ws[WS_SINV].ptr;
    float *theta = Theta_out ? Theta_out : (float *)ctx->ws[WS_THETA].ptr;
    float *z = (float *)ctx->ws[WS_SVOL].ptr;
    // TwIST rotates three iterate buffers: the new iterate never overwrites
    // one that the same kernel reads
    float *xa = X_out, *xb = (float *)ctx->ws[WS_XTMP].ptr, *xc = twist ? (float *)ctx->ws[WS_XNEXT].ptr : nullptr;
    auto rotate = [&]() { // x^(t+1) was written to xc
        float *old_b = xb;
        xb = xa;
        xa = xc;
        xc = old_b;
    };
    sci_tv_params q = p->tv;
    q.lambda = (float)((double)p->tv.lambda / L);
    {
        ProfScope prof(ctx, PF_SETUP, s);
        launch_fill(W, (float)(1.0 / L), img_elems(d), s);
        launch_pack_masks(d.nx, d.ny, d.B, C, cbits_ptr(ctx), cflag_ptr(ctx, d), s);
        if (X_init) launch_copy(X_init, xa, vb, s); // x^(0)
        else launch_adjoint(d.nx, d.ny, d.B, C, Y, xa, s);
        launch_copy(xa, theta, vb, s);
    }
    if ((st = check_launch(ctx, "setup")) != SCI_OK) return st;
    FgpRun r;
    bind_duals(ctx, r);
    const void *warm = nullptr; // warm_dual: the previous prox call's final dual
    double tau = 1.0;
    float ex = 0.0f; // FISTA: theta = xa + ex (xa - xb), formed by the projection as it loads
    const float a0 = (float)(1.0 - alpha), a1 = (float)(alpha - beta), a2 = (float)beta;
    bool pend = false; // TwIST: x^(t+1) = a0 xb + a1 xa + a2 theta not formed yet
    for (int t = 0; t < p->outer_iters; ++t) {
        {
            ProfScope prof(ctx, PF_PROJECT, s);
            // FISTA steps from the extrapolated point (x^(0) itself at first),
            // TwIST from x^(t), formed here (into the third buffer) once t >= 2
            if (!twist && t > 0) {
                launch_fista_project(d.nx, d.ny, d.B, xa, xb, ex, C, Y, W, z, s, cbits_ptr(ctx), cflag_ptr(ctx, d));
            } else if (pend) {
                launch_twist_project(d.nx, d.ny, d.B, xa, xb, theta, a0, a1, a2, C, Y, W, z, xc, s, cbits_ptr(ctx),
                                     cflag_ptr(ctx, d));
                rotate();
                pend = false;
            } else {
                launch_gap_project(d.nx, d.ny, d.B, xa, C, Y, W, z, s, cbits_ptr(ctx), cflag_ptr(ctx, d));
            }
        }
        if ((st = check_launch(ctx, "k_project")) != SCI_OK) return st;
        if (!twist) {
            // x^(t) into the other buffer; x^(t-1) stays in xa
            if ((st = denoise_fixed(ctx, d, q, z, xb, nullptr, warm, p->warm_dual != 0, r, s)) != SCI_OK) return st;
            const double tau1 = (1.0 + std::sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
            ex = (float)((tau - 1.0) / tau1);
            tau = tau1;
        } else {
            if ((st = denoise_fixed(ctx, d, q, z, theta, nullptr, warm, p->warm_dual != 0, r, s)) != SCI_OK) return st;
            if (t == 0) {
                launch_copy(theta, xb, vb, s); // x^(1) = theta^(0)
                std::swap(xa, xb);
            } else {
                pend = true; // the next projection (or the end of the loop) forms x^(t+1)
            }
        }
        if ((st = check_launch(ctx, "update")) != SCI_OK) return st;
        if (p->warm_dual) warm = r.cur;
        if (!twist) std::swap(xa, xb); // xa = newest iterate, xb = the one before
    }
    if (pend) {
        launch_two_step(V, a0, a1, a2, xb, xa, theta, xc, s);
        rotate();
    }
    // FISTA's last extrapolated point is stored only for the caller
    if (!twist && p->outer_iters > 0 && Theta_out) launch_extrapolate(V, ex, xa, xb, theta, s);
    if (xa != X_out) launch_copy(xa, X_out, vb, s);
    return check_launch(ctx, "copy");
}


// `n` more inner iterations of a gap-controlled denoiser call: on-chip passes
// of up to kTileMaxM iterations where the fused schedule applies, else one
// pass per iteration. The dual stays in r.cur for the gap check.
int fgp_chunk(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &q, const float *x, FgpRun &r, int n, hipStream_t s)
{
    const bool fused = q.schedule != SCI_SCHED_STREAM && fused_supported(q, d);
    if (q.schedule == SCI_SCHED_FUSED && !fused) return fail(ctx, SCI_ERR_UNSUPPORTED, kFusedScope);
    if (fused)
        return fgp_tile_iterate(ctx, d, q, x, r, n, nullptr, nullptr, true, s, -1, (n + kTileMaxM - 1) / kTileMaxM);
    return fgp_iterate(ctx, d, q, x, r, n, s);
}

// Denoise with a duality-gap stopping rule (relative gap <= q.gap_tol checked
// every q.gap_check_every iterations, at most q.n_inner_max), starting from
// `init` (nullable = zero dual). Leaves p in r.cur, writes theta, adds the
// iterations run to *iters and reports convergence.
int denoise_adaptive(sci_ctx *ctx, const sci_dims &d, const sci_tv_params &q, const float *x, float *theta,
                     float *u_out, const void *init, FgpRun &r, int *iters, bool *converged, hipStream_t s)
{
    const int every = q.gap_check_every > 0 ? q.gap_check_every : 10;
    r.cur = init;
    r.prev = nullptr;
    r.iters = 0;
    r.beta_prev = 0.0;
    r.mom = Momentum();
    *converged = false;
    int st = SCI_OK;
    double gap = 0.0, primal = 0.0;
    while (r.iters < q.n_inner_max) {
        const int n = std::min(every, q.n_inner_max - r.iters);
        if ((st = fgp_chunk(ctx, d, q, x, r, n, s)) != SCI_OK) return st;
        if ((st = rel_gap(ctx, d, q.tv, q.dual_dtype, q.lambda, x, r.cur, &gap, &primal, s)) != SCI_OK) return st;
        const double rel = relative_gap(gap, primal);
        if (gap_met(rel, q.gap_tol)) {
            *converged = true;
            break;
        }
        if (std::isnan(rel)) break; // a non-finite start does not recover: stop and report it
    }
    *iters += r.iters;
    st = launch_tv_theta(q.dual_dtype, d.nx, d.ny, d.B, x, r.cur, q.lambda, theta, u_out, s);
    if (st != SCI_OK) return fail(ctx, st, "theta pass");
    return check_launch(ctx, "k_tv_theta");
}

} // namespace
} // namespace sci

using namespace sci;

extern "C" {

int sci_forward(sci_ctx *ctx, sci_dims d, const float *C, const float *X, float *Y, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!C || !X || !Y) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    const size_t vb = vol_elems(d) * sizeof(float), ib = img_elems(d) * sizeof(float);
    if (overlaps(Y, ib, C, vb) || overlaps(Y, ib, X, vb)) return fail(ctx, SCI_ERR_ALIAS, "Y overlaps C or X");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    launch_forward(d.nx, d.ny, d.B, C, X, Y, stream);
    return check_launch(ctx, "k_forward");
}

int sci_adjoint(sci_ctx *ctx, sci_dims d, const float *C, const float *Y, float *X, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!C || !X || !Y) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    const size_t vb = vol_elems(d) * sizeof(float), ib = img_elems(d) * sizeof(float);
    if (overlaps(X, vb, C, vb) || overlaps(X, vb, Y, ib)) return fail(ctx, SCI_ERR_ALIAS, "X overlaps C or Y");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    launch_adjoint(d.nx, d.ny, d.B, C, Y, X, stream);
    return check_launch(ctx, "k_adjoint");
}

int sci_tv_denoise(sci_ctx *ctx, sci_dims d, const sci_tv_params *p, const float *X_in, float *Theta_out,
                   const void *dual_init, void *dual_out, double *rel_gap_out, int32_t *iters_out,
                   hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!p || !X_in || !Theta_out) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    if ((st = check_tv(ctx, *p, d)) != SCI_OK) return st;
    const bool adaptive = p->gap_tol > 0.0;
    if (adaptive && (p->n_inner_max < 1 || !std::isfinite(p->gap_tol)))
        return fail(ctx, SCI_ERR_INVALID_ARG, "gap_tol > 0 needs n_inner_max >= 1");
    const size_t vb = vol_elems(d) * sizeof(float);
    const size_t db = 2 * vol_elems(d) * dual_elem_bytes(p->dual_dtype);
    if (overlaps(Theta_out, vb, X_in, vb) || overlaps(Theta_out, vb, dual_init, db) ||
        overlaps(dual_out, db, X_in, vb) || overlaps(dual_out, db, dual_init, db) ||
        overlaps(dual_out, db, Theta_out, vb))
        return fail(ctx, SCI_ERR_ALIAS, "outputs must not overlap the inputs or each other");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    if ((st = ensure_duals(ctx, d, p->dual_dtype, stream, p)) != SCI_OK) return st;

    sci_tv_params q = *p;
    const bool want_dual = dual_out || rel_gap_out || adaptive;
    FgpRun r;
    bind_duals(ctx, r);

    if (q.lambda == 0.0f) {
        launch_copy(X_in, Theta_out, vb, stream);
        if (dual_out) {
            if (dual_init) launch_copy(dual_init, dual_out, db, stream);
            else launch_zero(dual_out, db, stream);
        }
        if ((st = check_launch(ctx, "copy")) != SCI_OK) return st;
        if (rel_gap_out) *rel_gap_out = 0.0;
        if (iters_out) *iters_out = 0;
        if (rel_gap_out) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
        }
        return SCI_OK;
    }

    int status = SCI_OK;
    double gap = 0.0, primal = 0.0;
    if (!adaptive) {
        if ((st = denoise_fixed(ctx, d, q, X_in, Theta_out, nullptr, dual_init, want_dual, r, stream)) != SCI_OK)
            return st;
        if (rel_gap_out) {
            if ((st = rel_gap(ctx, d, q.tv, q.dual_dtype, q.lambda, X_in, r.cur, &gap, &primal, stream)) != SCI_OK)
                return st;
        }
    } else {
        const int every = q.gap_check_every > 0 ? q.gap_check_every : 10;
        r.cur = dual_init;
        status = SCI_NOT_CONVERGED;
        while (r.iters < q.n_inner_max) {
            const int n = std::min(every, q.n_inner_max - r.iters);
            if ((st = fgp_chunk(ctx, d, q, X_in, r, n, stream)) != SCI_OK) return st;
            if ((st = rel_gap(ctx, d, q.tv, q.dual_dtype, q.lambda, X_in, r.cur, &gap, &primal, stream)) != SCI_OK)
                return st;
            const double rel = relative_gap(gap, primal);
            if (gap_met(rel, q.gap_tol)) {
                status = SCI_OK;
                break;
            }
            if (std::isnan(rel)) break; // non-finite gap: SCI_NOT_CONVERGED without running to the cap
        }
        st = launch_tv_theta(q.dual_dtype, d.nx, d.ny, d.B, X_in, r.cur, q.lambda, Theta_out, nullptr, stream);
        if (st == SCI_OK) st = check_launch(ctx, "k_tv_theta");
        if (st != SCI_OK) return st;
    }
    if (dual_out) {
        if (r.cur) launch_copy(r.cur, dual_out, db, stream);
        else launch_zero(dual_out, db, stream);
        if ((st = check_launch(ctx, "copy")) != SCI_OK) return st;
    }
    if (rel_gap_out) *rel_gap_out = relative_gap(gap, primal);
    if (iters_out) *iters_out = (q.n_inner == 0 && !adaptive) ? 0 : (adaptive ? r.iters : q.n_inner);
    return status;
}

int sci_gap_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
               float *Theta_out, const float *X_init, hipStream_t stream)
{
    return run_outer(ctx, d, p, Y, C, X_out, Theta_out, X_init, false, stream);
}

int sci_admm_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
                float *Theta_out, const float *X_init, hipStream_t stream)
{
    return run_outer(ctx, d, p, Y, C, X_out, Theta_out, X_init, true, stream);
}

int sci_gap_tv_noalloc(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
                       float *X_out, float *Theta_out, const float *X_init, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (img_elems(d) > kNoAllocMaxPixels)
        return fail(ctx, SCI_ERR_INVALID_ARG, "nx * ny exceeds the fixed scratch of the allocation-free GAP (4194304 pixels)");
    if ((st = check_outer_args(ctx, d, p, Y, C, X_out, Theta_out, X_init)) != SCI_OK) return st;
    if (!Theta_out) return fail(ctx, SCI_ERR_INVALID_ARG, "Theta_out is required (no scratch volume is allocated)");
    if (p->use_graph || p->warm_dual)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "the allocation-free GAP needs use_graph = 0 and warm_dual = 0");
    if (!ctx->noalloc_scratch) return fail(ctx, SCI_ERR_HIP, "fixed scratch address unknown");
    // every denoiser call is one cold on-chip pass that stores no dual field,
    // so the dual storage type does not change the result
    sci_solver_params q = *p;
    sci_tv_params &t = q.tv;
    t.dual_dtype = SCI_DUAL_F32;
    t.schedule = SCI_SCHED_FUSED;
    t.tile_passes = 1;
    if (t.lambda > 0.0f && t.n_inner > 0) {
        const int max_m = (t.tv == SCI_TV_VTV && !t.clip) ? vtv_rows_max_pass(d.B) : kTileMaxM;
        if (t.n_inner > max_m || !fused_supported(t, d))
            return fail(ctx, SCI_ERR_UNSUPPORTED,
                        "the allocation-free GAP runs each denoiser call in one on-chip pass (n_inner <= 10; "
                        "VTV: 10 / 10 / 7 / 4 for B <= 8 / 16 / 24 / 32)");
    }
    // no context event may be created here: the profiler is off for this call
    struct ProfOff {
        sci_ctx *c;
        bool was;
        ~ProfOff() { c->prof_on = was; }
    } prof_off{ctx, ctx->prof_on};
    ctx->prof_on = false;
    char *base = (char *)ctx->noalloc_scratch;
    OuterArgs a{d, q, Y, C, X_init, X_out, Theta_out, false, (float *)base, (uint32_t *)(base + kNoAllocBitsOffset),
                (int *)(base + kNoAllocFlagOffset), nullptr, nullptr, {nullptr, nullptr, nullptr, nullptr}};
    return enqueue_outer(ctx, a, stream);
}

int sci_fista_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
                 float *Theta_out, const float *X_init, hipStream_t stream)
{
    return run_prox_grad(ctx, d, p, Y, C, X_out, Theta_out, X_init, false, stream);
}

int sci_twist_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
                 float *Theta_out, const float *X_init, hipStream_t stream)
{
    return run_prox_grad(ctx, d, p, Y, C, X_out, Theta_out, X_init, true, stream);
}

int sci_gap_tv_adaptive(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
                        float *X_out, float *Theta_out, const float *X_init, sci_wsnet *net, int32_t *inner_iters_out,
                        int32_t *fallbacks_out, int32_t *net_starts_out, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!p || !Y || !C || !X_out) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    if ((st = check_tv(ctx, p->tv, d)) != SCI_OK) return st;
    const sci_tv_params &t0 = p->tv;
    if (!(t0.gap_tol > 0.0) || !std::isfinite(t0.gap_tol) || t0.n_inner_max < 1 || t0.lambda <= 0.0f)
        return fail(ctx, SCI_ERR_INVALID_ARG, "adaptive GAP needs gap_tol > 0, n_inner_max >= 1, lambda > 0");
    if (t0.dual_dtype != SCI_DUAL_F32) return fail(ctx, SCI_ERR_UNSUPPORTED, "adaptive GAP stores float32 duals");
    if (p->outer_iters < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "outer_iters must be >= 0");
    const size_t vb = vol_elems(d) * sizeof(float), ib = img_elems(d) * sizeof(float);
    const void *ins[3] = {Y, C, X_init};
    const size_t inb[3] = {ib, vb, vb};
    for (int k = 0; k < 3; ++k)
        if (overlaps(X_out, vb, ins[k], inb[k]) || overlaps(Theta_out, vb, ins[k], inb[k]))
            return fail(ctx, SCI_ERR_ALIAS, "outputs must not overlap Y, C or X_init");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_SINV, ib, stream)) != SCI_OK) return st;
    if (!Theta_out && (st = ensure_ws(ctx, WS_THETA, vb, stream)) != SCI_OK) return st;
    if ((st = ensure_duals(ctx, d, SCI_DUAL_F32, stream, &p->tv)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_XTMP, 2 * vb, stream)) != SCI_OK) return st; // predicted dual
    float *theta = Theta_out ? Theta_out : (float *)ctx->ws[WS_THETA].ptr;
    float *Sinv = (float *)ctx->ws[WS_SINV].ptr;
    float *pred = (float *)ctx->ws[WS_XTMP].ptr;
    const sci_tv_params &q = t0;
    if ((st = ensure_ws(ctx, WS_CBITS, cbits_bytes(d), stream)) != SCI_OK) return st;
    launch_weights(d.nx, d.ny, d.B, C, 0.0f, Sinv, stream);
    launch_pack_masks(d.nx, d.ny, d.B, C, cbits_ptr(ctx), cflag_ptr(ctx, d), stream);
    if (X_init) launch_copy(X_init, theta, vb, stream);
    else launch_adjoint(d.nx, d.ny, d.B, C, Y, theta, stream);
    if (p->outer_iters == 0) launch_copy(theta, X_out, vb, stream);
    if ((st = check_launch(ctx, "adaptive setup")) != SCI_OK) return st;
    FgpRun r;
    bind_duals(ctx, r);
    int inner = 0, fallbacks = 0, net_starts = 0;
    const void *keep = nullptr;
    for (int t = 0; t < p->outer_iters; ++t) {
        launch_gap_project(d.nx, d.ny, d.B, theta, C, Y, Sinv, X_out, stream, cbits_ptr(ctx), cflag_ptr(ctx, d));
        if ((st = check_launch(ctx, "k_project")) != SCI_OK) return st;
        const void *init = nullptr;
        // a correcting network (3 input channels) needs the previous call's final dual,
        // so the first call starts cold
        const bool use_net = net && (wsnet_input_channels(net) == 1 || keep);
        if (use_net) {
            if ((st = sci_wsnet_forward(ctx, net, d, X_out, (const float *)keep, nullptr, q.tv, pred, stream)) !=
                SCI_OK)
                return st;
            init = pred;
            if (p->warm_dual && keep) {
                // gap-checked start: the prediction or the previous final dual,
                // whichever has the smaller relative duality gap on this input
                double gp = 0.0, pp = 0.0, gk = 0.0, pk = 0.0;
                if ((st = rel_gap(ctx, d, q.tv, q.dual_dtype, q.lambda, X_out, pred, &gp, &pp, stream)) != SCI_OK)
                    return st;
                if ((st = rel_gap(ctx, d, q.tv, q.dual_dtype, q.lambda, X_out, keep, &gk, &pk, stream)) != SCI_OK)
                    return st;
                // a non-finite gap loses: the prediction is taken only when its
                // gap is finite and no larger than the previous dual's
                const double rp = relative_gap(gp, pp), rk = relative_gap(gk, pk);
                if (std::isfinite(rp) && !(rk < rp)) ++net_starts;
                else init = keep;
            } else {
                ++net_starts;
            }
        } else if (p->warm_dual) {
            init = keep;
        }
        bool ok = false;
        if ((st = denoise_adaptive(ctx, d, q, X_out, theta, nullptr, init, r, &inner, &ok, stream)) != SCI_OK)
            return st;
        if (!ok && init == pred) { // the predicted start did not reach the tolerance: cold start
            ++fallbacks;
            if ((st = denoise_adaptive(ctx, d, q, X_out, theta, nullptr, nullptr, r, &inner, &ok, stream)) != SCI_OK)
                return st;
        }
        keep = r.cur;
    }
    if (inner_iters_out) *inner_iters_out = inner;
    if (fallbacks_out) *fallbacks_out = fallbacks;
    if (net_starts_out) *net_starts_out = net_starts;
    return SCI_OK;
}

int sci_tile_shape_count(void) { return tile_shape_count(); }

int sci_tile_shape_info(int32_t shape, int32_t *rows_per_wave, int32_t *waves_per_group, int32_t *cols_per_lane)
{
    int r = 0, w = 0, c = 0;
    if (!tile_shape_info(shape - 1, &r, &w, &c)) return SCI_ERR_INVALID_ARG;
    if (rows_per_wave) *rows_per_wave = r;
    if (waves_per_group) *waves_per_group = w;
    if (cols_per_lane) *cols_per_lane = c;
    return SCI_OK;
}

int sci_tile_shape_pipelined(int32_t shape)
{
    int r = 0, w = 0, c = 0;
    if (!tile_shape_info(shape - 1, &r, &w, &c)) return SCI_ERR_INVALID_ARG;
    return tile_shape_pipelined(shape - 1) ? 1 : 0;
}

int sci_autotune(sci_ctx *ctx, sci_dims d, const sci_tv_params *p, const float *X, int32_t *best_shape_out,
                 int32_t *best_passes_out, double *times_ms_out, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!p || !X) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    if ((st = check_tv(ctx, *p, d)) != SCI_OK) return st;
    if (!tile_supported(p->tv) || p->chambolle04 || p->clip)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "only the tiled FGP / projected-gradient denoiser (ATV, ITV2D) is tuned");
    if (p->lambda == 0.0f || p->n_inner == 0) return fail(ctx, SCI_ERR_INVALID_ARG, "nothing to tune: lambda or n_inner is 0");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    const size_t vb = vol_elems(d) * sizeof(float);
    if ((st = ensure_duals(ctx, d, p->dual_dtype, stream, p)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_THETA, vb, stream)) != SCI_OK) return st;
    float *theta = (float *)ctx->ws[WS_THETA].ptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, SCI_ERR_HIP, "hipEventCreate");
    const int nshape = tile_shape_count();
    const int n = p->n_inner;
    const int pmin = (n + kTileMaxM - 1) / kTileMaxM;
    const int reps = 3;
    int best_s = 0, best_p = pmin;
    double best_ms = 1e300;
    const bool one_per_pass = p->schedule == SCI_SCHED_STREAM;
    sci_tv_params q = *p;
    q.schedule = one_per_pass ? SCI_SCHED_STREAM : SCI_SCHED_FUSED;
    FgpRun r;
    bind_duals(ctx, r);
    for (int sh = 0; sh < nshape && st == SCI_OK; ++sh) {
        for (int k = 0; k < kTuneSplits && st == SCI_OK; ++k) {
            const int np = one_per_pass ? n : pmin + k;
            if (times_ms_out) times_ms_out[sh * kTuneSplits + k] = NAN;
            if (np > n || (one_per_pass && k > 0)) continue;
            q.tile_shape = sh + 1;
            q.tile_passes = np;
            st = denoise_fixed(ctx, d, q, X, theta, nullptr, nullptr, false, r, stream); // warm-up
            if (st == SCI_OK && hipEventRecord(e0, stream) != hipSuccess) st = fail(ctx, SCI_ERR_HIP, "hipEventRecord");
            for (int rep = 0; rep < reps && st == SCI_OK; ++rep)
                st = denoise_fixed(ctx, d, q, X, theta, nullptr, nullptr, false, r, stream);
            if (st != SCI_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(ctx, SCI_ERR_HIP, "autotune timing");
                break;
            }
            const double t = (double)ms / reps;
            if (times_ms_out) times_ms_out[sh * kTuneSplits + k] = t;
            if (t < best_ms) {
                best_ms = t;
                best_s = sh;
                best_p = np;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SCI_OK) return st;
    ctx->tuned[tune_key(q, d)] = std::make_pair(best_s, best_p);
    if ((st = drop_graphs(ctx)) != SCI_OK) return st;
    if (best_shape_out) *best_shape_out = best_s + 1;
    if (best_passes_out) *best_passes_out = best_p;
    return SCI_OK;
}

int sci_psnr(sci_ctx *ctx, int64_t count, const float *a, const float *ref, double peak, double *out_host,
             hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    if (count < 1 || !a || !ref || !out_host || !std::isfinite(peak) || peak <= 0.0)
        return fail(ctx, SCI_ERR_INVALID_ARG, "psnr: bad arguments");
    int st = use_device(ctx);
    if (st != SCI_OK) return st;
    const int nb = reduce_partial_blocks();
    if ((st = ensure_ws(ctx, WS_PARTIAL, (3 * (size_t)nb + 8) * sizeof(double), stream)) != SCI_OK) return st;
    double *part = (double *)ctx->ws[WS_PARTIAL].ptr;
    launch_sqdiff(count, a, ref, part, part + 3 * nb, stream);
    if ((st = check_launch(ctx, "k_sqdiff")) != SCI_OK) return st;
    if ((st = read_scalars(ctx, part + 3 * nb, 1, stream)) != SCI_OK) return st;
    const double mse = ctx->host_scalars[0] / (double)count;
    *out_host = 10.0 * std::log10(peak * peak / mse);
    return SCI_OK;
}

int sci_residual_sq(sci_ctx *ctx, sci_dims d, const float *C, const float *X, const float *Y, double *out_host,
                    hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!C || !X || !Y || !out_host) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    const int nb = reduce_partial_blocks();
    if ((st = ensure_ws(ctx, WS_PARTIAL, (3 * (size_t)nb + 8) * sizeof(double), stream)) != SCI_OK) return st;
    double *part = (double *)ctx->ws[WS_PARTIAL].ptr;
    launch_residual_sq(d.nx, d.ny, d.B, C, X, Y, part, part + 3 * nb, stream);
    if ((st = check_launch(ctx, "k_resid")) != SCI_OK) return st;
    if ((st = read_scalars(ctx, part + 3 * nb, 1, stream)) != SCI_OK) return st;
    *out_host = ctx->host_scalars[0];
    return SCI_OK;
}

int sci_dual_gap(sci_ctx *ctx, sci_dims d, int32_t tv, int32_t dual_dtype, float lambda, const float *X,
                 const void *p, double *gap_host, double *primal_host, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = check_dims(ctx, d);
    if (st != SCI_OK) return st;
    if (!X || !p) return fail(ctx, SCI_ERR_INVALID_ARG, "null pointer argument");
    if (tv < SCI_TV_ATV || tv > SCI_TV_VTV || dual_dtype < SCI_DUAL_F32 || dual_dtype > SCI_DUAL_F16 ||
        !std::isfinite(lambda) || lambda < 0.0f)
        return fail(ctx, SCI_ERR_INVALID_ARG, "dual_gap: bad tv, dtype or lambda");
    if ((st = use_device(ctx)) != SCI_OK) return st;
    double gap = 0.0, primal = 0.0;
    if ((st = rel_gap(ctx, d, tv, dual_dtype, lambda, X, p, &gap, &primal, stream)) != SCI_OK) return st;
    if (gap_host) *gap_host = gap;
    if (primal_host) *primal_host = primal;
    return SCI_OK;
}

} // extern "C"
