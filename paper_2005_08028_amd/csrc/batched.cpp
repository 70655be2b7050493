// Host driver of the batched GAP-TV solve: many independent measurements of
// different sizes reconstructed together, one batched projection and one
// batched fused-denoise launch per outer iteration (VTV: one row-pipelined
// pass per problem still iterating), the whole loop captured once in a HIP
// graph.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "sci_batched.h"
#include "sci_internal.h"

namespace sci {
namespace {

constexpr int kPixBlock = 256;

struct BatchPlan {
    std::vector<BatchProb> tab; // sorted by descending outer_iters
    std::vector<int> order;     // tab[k] is problem order[k]
    std::vector<int> wg_end;    // wg_end[k] = workgroups of problems 0..k-1 (prefix)
    std::vector<int> pb_end;
    std::vector<int> pj_end;
    int maxB = 0, Tmax = 0, shape = 0, m = 0;
    size_t slab_floats = 0;
};

std::string batch_key(const sci_solver_params &p, int n, const sci_problem *probs)
{
    std::string k = "batch|" + std::to_string(p.tv.tv) + "|" + std::to_string(p.tv.n_inner);
    for (int i = 0; i < n; ++i)
        k += "|" + std::to_string(probs[i].d.nx) + "x" + std::to_string(probs[i].d.ny) + "x" +
             std::to_string(probs[i].d.B);
    return k;
}

int validate(sci_ctx *ctx, int n, const sci_problem *probs, const sci_solver_params *p)
{
    if (n < 1 || !probs || !p) return fail(ctx, SCI_ERR_INVALID_ARG, "batched: n >= 1, probs and params required");
    const sci_tv_params &t = p->tv;
    if (t.tv != SCI_TV_ATV && t.tv != SCI_TV_ITV2D && t.tv != SCI_TV_VTV)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "batched solve covers ATV, ITV2D and VTV (fused schedule)");
    if (!std::isfinite(t.lambda) || t.lambda <= 0.0f) return fail(ctx, SCI_ERR_INVALID_ARG, "batched: lambda must be > 0");
    if (t.n_inner < 1 || t.n_inner > kTileMaxM)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "batched: n_inner must be in 1..10 (one on-chip pass)");
    if (t.accel != 0 && t.accel != 1) return fail(ctx, SCI_ERR_INVALID_ARG, "accel must be 0 or 1");
    if (t.tile_shape < 0 || t.tile_shape > tile_shape_count())
        return fail(ctx, SCI_ERR_INVALID_ARG, "tile_shape out of range");
    if (p->outer_iters < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "outer_iters must be >= 0");
    if (p->warm_dual) return fail(ctx, SCI_ERR_UNSUPPORTED, "batched: cold-start denoiser only");
    if (t.chambolle04 || t.clip)
        return fail(ctx, SCI_ERR_UNSUPPORTED, "batched: FGP / projected-gradient denoiser only");
    for (int i = 0; i < n; ++i) {
        const sci_problem &q = probs[i];
        if (q.d.nx < 1 || q.d.ny < 1 || q.d.B < 1 || (int64_t)q.d.nx * q.d.ny * q.d.B >= ((int64_t)1 << 31))
            return fail(ctx, SCI_ERR_INVALID_ARG, "batched: bad dims of problem " + std::to_string(i));
        if (q.d.B > 32) return fail(ctx, SCI_ERR_UNSUPPORTED, "batched: B <= 32 per problem");
        // VTV: the denoise is one cold pass of the length a lone solve would
        // also run unsplit, so the dual never leaves the chip
        if (t.tv == SCI_TV_VTV && t.n_inner > vtv_rows_auto_pass(q.d.B, true))
            return fail(ctx, SCI_ERR_UNSUPPORTED,
                        "batched VTV: n_inner must fit one pass, at most " +
                            std::to_string(vtv_rows_auto_pass(q.d.B, true)) + " iterations for B = " +
                            std::to_string(q.d.B) + " (problem " + std::to_string(i) + ")");
        if (!q.Y || !q.C || !q.X_out) return fail(ctx, SCI_ERR_INVALID_ARG, "batched: null pointer in problem " + std::to_string(i));
        if (q.outer_iters < 0) return fail(ctx, SCI_ERR_INVALID_ARG, "batched: outer_iters must be >= 0");
        const size_t vb = (size_t)q.d.nx * q.d.ny * q.d.B * 4, ib = (size_t)q.d.nx * q.d.ny * 4;
        if (overlaps(q.X_out, vb, q.Y, ib) || overlaps(q.X_out, vb, q.C, vb) || overlaps(q.Theta_out, vb, q.Y, ib) ||
            overlaps(q.Theta_out, vb, q.C, vb) || overlaps(q.X_out, vb, q.Theta_out, vb))
            return fail(ctx, SCI_ERR_ALIAS, "batched: outputs overlap inputs in problem " + std::to_string(i));
    }
    return SCI_OK;
}

void plan_batch(const sci_ctx *ctx, int n, const sci_problem *probs, const sci_solver_params &p, int shape_override,
                BatchPlan &pl)
{
    pl.m = p.tv.n_inner;
    pl.shape = 0;
    auto it = ctx->tuned.find(batch_key(p, n, probs));
    if (it != ctx->tuned.end()) pl.shape = it->second.first;
    if (p.tv.tile_shape >= 1) pl.shape = p.tv.tile_shape - 1;
    if (shape_override >= 0) pl.shape = shape_override;
    int tw = 0, th = 0;
    batch_tile_extent(pl.shape, pl.m, &tw, &th);
    pl.order.resize(n);
    std::iota(pl.order.begin(), pl.order.end(), 0);
    auto T = [&](int i) { return probs[i].outer_iters > 0 ? probs[i].outer_iters : p.outer_iters; };
    std::stable_sort(pl.order.begin(), pl.order.end(), [&](int a, int b) { return T(a) > T(b); });
    pl.tab.assign(n, BatchProb{});
    pl.wg_end.assign(n + 1, 0);
    pl.pb_end.assign(n + 1, 0);
    pl.pj_end.assign(n + 1, 0);
    pl.slab_floats = 0;
    pl.maxB = 0;
    pl.Tmax = 0;
    for (int k = 0; k < n; ++k) {
        const sci_problem &q = probs[pl.order[k]];
        BatchProb &b = pl.tab[k];
        b.nx = q.d.nx;
        b.ny = q.d.ny;
        b.B = q.d.B;
        b.outer_iters = T(pl.order[k]);
        b.ntx = (q.d.ny + tw - 1) / tw;
        b.ntiles = b.ntx * ((q.d.nx + th - 1) / th);
        b.wg_base = pl.wg_end[k];
        b.pb_base = pl.pb_end[k];
        pl.wg_end[k + 1] = b.wg_base + b.ntiles * b.B;
        const int npix = q.d.nx * q.d.ny;
        pl.pb_end[k + 1] = b.pb_base + (npix + kPixBlock - 1) / kPixBlock;
        auto al8 = [](const void *ptr) { return ptr == nullptr || ((uintptr_t)ptr & 7u) == 0; };
        b.pairs = npix % 2 == 0 && al8(q.Y) && al8(q.C) && al8(q.X_out) && al8(q.Theta_out) ? 1 : 0;
        b.pj_base = pl.pj_end[k];
        const int units = b.pairs ? npix / 2 : npix;
        pl.pj_end[k + 1] = b.pj_base + (units + kPixBlock - 1) / kPixBlock;
        b.Y = q.Y;
        b.C = q.C;
        b.x = q.X_out;
        b.theta = q.Theta_out;
        pl.slab_floats += 2 * (((size_t)npix + 63) & ~(size_t)63) + 64; // Sinv, mask bits, flag
        if (!q.Theta_out) pl.slab_floats += ((size_t)npix * q.d.B + 63) & ~(size_t)63;
        pl.maxB = std::max(pl.maxB, b.B);
        pl.Tmax = std::max(pl.Tmax, b.outer_iters);
    }
}

void bind_slab(float *slab, BatchPlan &pl)
{
    size_t off = 0;
    for (BatchProb &b : pl.tab) {
        const size_t npix = (size_t)b.nx * b.ny;
        b.Sinv = slab + off;
        off += (npix + 63) & ~(size_t)63;
        b.cbits = (uint32_t *)(slab + off);
        off += (npix + 63) & ~(size_t)63;
        b.cflag = (int *)(slab + off);
        off += 64;
        if (!b.theta) {
            b.theta = slab + off;
            off += (npix * b.B + 63) & ~(size_t)63;
        }
    }
}

int active_count(const BatchPlan &pl, int t)
{
    int k = 0;
    while (k < (int)pl.tab.size() && pl.tab[k].outer_iters > t) ++k;
    return k;
}

int enqueue_batch(sci_ctx *ctx, const BatchPlan &pl, const BatchProb *tab_dev, const sci_solver_params &p,
                  hipStream_t s)
{
    const int n = (int)pl.tab.size();
    {
        ProfScope prof(ctx, PF_SETUP, s);
        launch_batch_setup(n, pl.pb_end[n], tab_dev, s);
    }
    int st = check_launch(ctx, "k_batch_setup");
    if (st != SCI_OK) return st;
    TileBeta bt{};
    double nu = 1.0;
    for (int t = 0; t < pl.m; ++t) {
        const double nu1 = (1.0 + std::sqrt(1.0 + 4.0 * nu * nu)) / 2.0;
        bt.b[t + 1] = p.tv.accel ? (float)((nu - 1.0) / nu1) : 0.0f;
        nu = nu1;
    }
    for (int t = 0; t < pl.Tmax; ++t) {
        const int na = active_count(pl, t);
        {
            ProfScope prof(ctx, PF_PROJECT, s);
            st = launch_batch_project(na, pl.pj_end[na], pl.maxB, tab_dev, s);
        }
        if (st != SCI_OK) return fail(ctx, st, "batched projection");
        if ((st = check_launch(ctx, "k_batch_project")) != SCI_OK) return st;
        if (p.tv.tv == SCI_TV_VTV) {
            ProfScope prof(ctx, PF_FGP_FUSED, s);
            for (int k = 0; k < na && st == SCI_OK; ++k) {
                const BatchProb &b = pl.tab[k];
                TilePass tp; // cold start, theta out; the dual stays on chip
                tp.mode = 0;
                tp.beta = bt;
                tp.theta = b.theta;
                st = launch_vtv_rows(pl.m, b.nx, b.ny, b.B, b.x, tp, p.tv.lambda, s);
            }
        } else {
            ProfScope prof(ctx, PF_FGP_FUSED, s);
            st = launch_batch_denoise(p.tv.tv, pl.shape, pl.m, na, pl.wg_end[na], tab_dev, bt, p.tv.lambda, s);
        }
        if (st != SCI_OK) return fail(ctx, st, "batched denoise");
        if ((st = check_launch(ctx, "k_batch_denoise")) != SCI_OK) return st;
    }
    return SCI_OK;
}

int upload_table(sci_ctx *ctx, const BatchPlan &pl, BatchProb *dst, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, pl.tab.data(), pl.tab.size() * sizeof(BatchProb), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipMemcpyAsync(batch table)");
    e = hipStreamSynchronize(s); // the host copy of the table dies with this call
    if (e != hipSuccess) return fail_hip(ctx, e, "hipStreamSynchronize");
    return SCI_OK;
}

} // namespace
} // namespace sci

using namespace sci;

extern "C" {

int sci_gap_tv_batched(sci_ctx *ctx, int32_t n, const sci_problem *probs, const sci_solver_params *p,
                       hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = validate(ctx, n, probs, p);
    if (st != SCI_OK) return st;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipSetDevice");
    }
    BatchPlan pl;
    plan_batch(ctx, n, probs, *p, -1, pl);
    if ((st = ensure_ws(ctx, WS_BATCH, pl.slab_floats * sizeof(float), stream)) != SCI_OK) return st;
    bind_slab((float *)ctx->ws[WS_BATCH].ptr, pl);

    if (!p->use_graph) {
        if ((st = ensure_ws(ctx, WS_BDESC, pl.tab.size() * sizeof(BatchProb), stream)) != SCI_OK) return st;
        BatchProb *tab = (BatchProb *)ctx->ws[WS_BDESC].ptr;
        if ((st = upload_table(ctx, pl, tab, stream)) != SCI_OK) return st;
        return enqueue_batch(ctx, pl, tab, *p, stream);
    }
    // graph: keyed by every pointer and size of the batch; owns its own table
    std::string key = "batched|" + batch_key(*p, n, probs) + "|" + std::to_string(pl.shape) + "|" +
                      std::to_string(p->outer_iters) + "|" + std::to_string(p->tv.lambda) + "|" +
                      std::to_string(p->tv.accel);
    char buf[64];
    for (const BatchProb &b : pl.tab) {
        snprintf(buf, sizeof buf, "|%p,%p,%p,%p,%d", (const void *)b.Y, (const void *)b.C, (void *)b.x,
                 (void *)b.theta, b.outer_iters);
        key += buf;
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        void *tab = nullptr;
        hipError_t e = hipMalloc(&tab, pl.tab.size() * sizeof(BatchProb));
        if (e != hipSuccess) return fail_hip(ctx, e, "hipMalloc(batch table)");
        if ((st = upload_table(ctx, pl, (BatchProb *)tab, stream)) != SCI_OK) {
            (void)hipFree(tab);
            return st;
        }
        e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipFree(tab);
            return fail_hip(ctx, e, "hipStreamBeginCapture");
        }
        ctx->capturing = true;
        st = enqueue_batch(ctx, pl, (BatchProb *)tab, *p, ctx->capture_stream);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->capture_stream, &g);
        if (st != SCI_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipFree(tab);
            return st != SCI_OK ? st : fail_hip(ctx, e, "hipStreamEndCapture");
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            (void)hipFree(tab);
            return fail_hip(ctx, e, "hipGraphInstantiate");
        }
        it = ctx->graphs.emplace(key, GraphEntry{exec, tab}).first;
    }
    hipError_t e = hipGraphLaunch(it->second.exec, stream);
    if (e != hipSuccess) return fail_hip(ctx, e, "hipGraphLaunch");
    return SCI_OK;
}

int sci_autotune_batched(sci_ctx *ctx, int32_t n, const sci_problem *probs, const sci_solver_params *p,
                         int32_t *best_shape_out, double *times_ms_out, hipStream_t stream)
{
    if (!ctx) return SCI_ERR_INVALID_ARG;
    int st = validate(ctx, n, probs, p);
    if (st != SCI_OK) return st;
    if (p->tv.tv == SCI_TV_VTV) return fail(ctx, SCI_ERR_UNSUPPORTED, "batched VTV has no tile shape to tune");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return fail_hip(ctx, e, "hipSetDevice");
    }
    BatchPlan pl;
    plan_batch(ctx, n, probs, *p, 0, pl);
    if ((st = ensure_ws(ctx, WS_BATCH, pl.slab_floats * sizeof(float), stream)) != SCI_OK) return st;
    if ((st = ensure_ws(ctx, WS_BDESC, pl.tab.size() * sizeof(BatchProb), stream)) != SCI_OK) return st;
    float *slab = (float *)ctx->ws[WS_BATCH].ptr;
    BatchProb *tab = (BatchProb *)ctx->ws[WS_BDESC].ptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, SCI_ERR_HIP, "hipEventCreate");
    TileBeta bt{};
    double nu = 1.0;
    for (int t = 0; t < pl.m; ++t) {
        const double nu1 = (1.0 + std::sqrt(1.0 + 4.0 * nu * nu)) / 2.0;
        bt.b[t + 1] = p->tv.accel ? (float)((nu - 1.0) / nu1) : 0.0f;
        nu = nu1;
    }
    int best = 0;
    double best_ms = 1e300;
    const int nshape = tile_shape_count();
    for (int sh = 0; sh < nshape && st == SCI_OK; ++sh) {
        plan_batch(ctx, n, probs, *p, sh, pl);
        bind_slab(slab, pl);
        // time the denoise of all problems on their first projection (outer_iters ignored)
        for (BatchProb &b : pl.tab) b.outer_iters = 1;
        const int nb = (int)pl.tab.size();
        if ((st = upload_table(ctx, pl, tab, stream)) != SCI_OK) break;
        launch_batch_setup(nb, pl.pb_end[nb], tab, stream);
        if ((st = launch_batch_project(nb, pl.pj_end[nb], pl.maxB, tab, stream)) != SCI_OK) break;
        const int reps = 3;
        for (int r = 0; r <= reps && st == SCI_OK; ++r) {
            if (r == 1 && hipEventRecord(e0, stream) != hipSuccess) st = fail(ctx, SCI_ERR_HIP, "hipEventRecord");
            if (st == SCI_OK) st = launch_batch_denoise(p->tv.tv, sh, pl.m, nb, pl.wg_end[nb], tab, bt, p->tv.lambda, stream);
        }
        if (st != SCI_OK) break;
        if ((st = check_launch(ctx, "autotune batched")) != SCI_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(ctx, SCI_ERR_HIP, "autotune timing");
            break;
        }
        const double t = (double)ms / reps;
        if (times_ms_out) times_ms_out[sh] = t;
        if (t < best_ms) {
            best_ms = t;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SCI_OK) return st;
    ctx->tuned[batch_key(*p, n, probs)] = std::make_pair(best, 1);
    if ((st = drop_graphs(ctx)) != SCI_OK) return st;
    if (best_shape_out) *best_shape_out = best + 1;
    return SCI_OK;
}

} // extern "C"
