/*
 * libscitv — GAP-TV / ADMM-TV reconstruction for snapshot video compressive
 * imaging (SCI) on AMD Instinct MI355X (gfx950).
 *
 * Method: X. Yuan, "Various Total Variation for Snapshot Video Compressive
 * Imaging", arXiv:2005.08028. Equation numbers below count the paper's
 * numbered displays in order of appearance.
 *
 * Measurement model (Eq. (1)-(5)): B frames X_k in R^{nx x ny} are coded by
 * masks C_k and summed into one image, Y = sum_k C_k .* X_k + G. Phi is never
 * formed: the caller passes the B mask images.
 *
 * Conventions for every entry point
 *   - Arrays are caller-owned DEVICE pointers (memory of the device the
 *     context was created on), contiguous, row-major, column index fastest:
 *       video  [B][nx][ny] float32          (frame k, row i, column j)
 *       image  [nx][ny]    float32
 *       dual   [2][B][nx][ny] in the dual storage type of the call
 *              (channel 0 = horizontal differences along j, 1 = vertical
 *              along i). Entries with no difference behind them (j = ny-1
 *              in channel 0, i = nx-1 in channel 1) are written as 0 and
 *              ignored on input.
 *   - The library never frees or retains caller memory. Scratch buffers,
 *     graphs and tables belong to the context.
 *   - Work is enqueued on `stream` (0 = the legacy default stream) and is
 *     asynchronous unless a host output is requested (then the call
 *     synchronises `stream` before returning).
 *   - Every call validates its arguments before launching anything and
 *     returns a status code; no C++ exception crosses this interface.
 *     Outputs must not overlap inputs (SCI_ERR_ALIAS).
 *   - Sizes: nx, ny, B >= 1, B <= 65535 and B*nx*ny < 2^31.
 *   - Array values are expected finite; the library does not scan them, and
 *     a NaN or infinity in an input spreads through the result (it may also
 *     reach entries a finite input would leave at 0).
 *   - A context may be used from one host thread at a time. Calls that
 *     share a context and overlap on different streams race on its scratch.
 */
#ifndef SCITV_H
#define SCITV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SCI_OK 0
#define SCI_NOT_CONVERGED 1     /* outputs written; the duality-gap tolerance was not met at the cap */
#define SCI_ERR_INVALID_ARG (-1)/* null pointer, size out of range, lambda/rho < 0 or non-finite, bad enum */
#define SCI_ERR_ALIAS (-2)      /* an output overlaps an input */
#define SCI_ERR_NOMEM (-3)      /* device scratch allocation failed */
#define SCI_ERR_HIP (-4)        /* a HIP runtime call failed; sci_last_error() has the text */
#define SCI_ERR_UNSUPPORTED (-5)/* valid request the library does not implement (message in sci_last_error) */

typedef struct sci_ctx sci_ctx;

typedef struct {
    int32_t nx; /* rows i    */
    int32_t ny; /* columns j */
    int32_t B;  /* frames k  */
} sci_dims;

/* TV regulariser (Sec. 2.1). ITV2D and ITV3D are per-pixel isotropic norms:
 * ITV2D over (h, v) of one voxel (Eq. (9), dual projection Eq. (29)-(30));
 * SCI_TV_VTV is the paper's ITV3D, a norm over (h, v) of all B frames at one
 * pixel (Eq. (10), dual projection Eq. (31)-(32)); all frames of a pixel are
 * held by one workgroup, so VTV takes B <= 48 (B <= 32 on the fused
 * schedule, more on the streaming one; otherwise SCI_ERR_UNSUPPORTED). */
typedef enum { SCI_TV_ATV = 0, SCI_TV_ITV2D = 1, SCI_TV_VTV = 2 } sci_tv_kind;

/* Storage type of the dual fields kept in device memory between denoiser
 * passes; arithmetic is always float32. */
typedef enum { SCI_DUAL_F32 = 0, SCI_DUAL_BF16 = 1, SCI_DUAL_F16 = 2 } sci_dual_dtype;

/* How the inner denoiser iterations are scheduled on the GPU:
 *   STREAM: one pass over HBM per inner iteration (dual fields in memory);
 *   FUSED : up to 10 inner iterations per on-chip pass, the dual fields
 *           written back only between passes (ATV and ITV2D with any dual
 *           type; VTV with any dual type, passes of at most 10 / 10 / 7 / 4
 *           iterations for B <= 8 / 16 / 24 / 32; the Chambolle-2004 step
 *           with float32 duals on the row-pipelined kernels; ATV-Clip with
 *           float32 duals);
 *   AUTO  : FUSED where it applies, else STREAM.
 * Both schedules evaluate the same per-voxel expressions (bit for bit with
 * float32 duals; 16-bit duals are rounded where they are stored: after every
 * iteration on STREAM, between passes on FUSED). */
typedef enum { SCI_SCHED_AUTO = 0, SCI_SCHED_STREAM = 1, SCI_SCHED_FUSED = 2 } sci_schedule;

/* TV denoiser parameters: theta = argmin 1/2 ||theta - x||^2 + lambda TV(theta)
 * solved on the dual with step 1/(8 lambda) (Algorithm 1, FGP box). */
typedef struct {
    int32_t tv;              /* sci_tv_kind */
    float lambda;            /* TV weight >= 0; 0 returns the input unchanged */
    int32_t n_inner;         /* inner iterations (In-Iter) >= 0; 0 returns the input */
    int32_t accel;           /* 1 = FGP (Beck-Teboulle momentum), 0 = Chambolle projected gradient */
    int32_t dual_dtype;      /* sci_dual_dtype */
    int32_t schedule;        /* sci_schedule */
    double gap_tol;          /* sci_tv_denoise only: > 0 iterates until the relative duality
                                gap <= gap_tol (checked every gap_check_every iterations,
                                at most n_inner_max iterations; on the fused schedule the
                                iterations between two checks run in on-chip passes of up to
                                10); <= 0 runs exactly n_inner. With 16-bit dual storage the
                                gap is that of the stored dual, which rounding may move out of
                                the unit ball by half an ulp: its gap can then come out at or
                                slightly below zero and meet any tolerance, so tolerances
                                below what the storage type resolves certify nothing more */
    int32_t n_inner_max;
    int32_t gap_check_every;
    int32_t tile_shape;      /* fused schedule: 0 = autotuned for this problem (sci_autotune) or the
                                default (a cold call of at most 10 iterations whose dual is not
                                returned: the row-pipelined shape that best fills the GPU when
                                the problem is large enough; otherwise shape 1); k >= 1 = shape k
                                (see sci_tile_shape_info) */
    int32_t tile_passes;     /* fused schedule: passes over HBM per denoiser call (each runs about
                                n_inner / tile_passes iterations, at most 10); 0 = autotuned or
                                default (passes of about 5 iterations; VTV: the fewest passes its
                                kernel runs) */
    int32_t chambolle04;     /* 1 = Chambolle's (2004) semi-implicit step (Sec. 2.3):
                                p = (w + z/(8 lambda)) / (1 + |z|/(8 lambda)), z = D theta, |z| per
                                the TV kind, in place of the projection of w + z/(8 lambda);
                                fused schedule (float32 duals): row-pipelined passes (for ATV
                                and ITV2D tile_shape is then a row-pipelined shape or 0);
                                16-bit duals run on the streaming schedule (AUTO picks it;
                                FUSED is SCI_ERR_UNSUPPORTED). 0 = projection */
    int32_t clip;            /* 1 = ATV-Clip (Sec. 2.3, Algorithm 1 Clip box): one dual per
                                direction, w_d <- clip(w_d + D_d (x - D_d^T w_d) / clip_alpha,
                                2 lambda), output x - D_h^T w_h - D_v^T w_v; tv must be ATV,
                                fixed n_inner (accel and chambolle04 do not apply); fused
                                schedule (float32 duals): row-pipelined passes (tile_shape a
                                row-pipelined shape or 0); 16-bit duals run on the streaming
                                schedule (AUTO picks it; FUSED is SCI_ERR_UNSUPPORTED).
                                0 = FGP / projected gradient */
    float clip_alpha;        /* ATV-Clip step 1/clip_alpha; 0 = 4 (the largest eigenvalue of
                                D_d D_d^T is below 4; the iteration converges for alpha > 2) */
} sci_tv_params;

/* Outer framework parameters (Algorithm 1; ADMM of Eq. (24)-(26)). */
typedef struct {
    sci_tv_params tv;        /* denoiser used once per outer iteration (fixed n_inner) */
    int32_t outer_iters;     /* MaxIter >= 0 */
    float rho;               /* ADMM penalty >= 0 (ignored by GAP) */
    int32_t warm_dual;       /* 1 = carry the denoiser's dual from one outer iteration to
                                the next (momentum restarted), 0 = cold start every call */
    int32_t use_graph;       /* 1 = capture the outer loop once in a HIP graph and replay it */
    float twist_alpha;       /* TwIST two-step weights; both 0 = the values the spectrum-bound */
    float twist_beta;        /* formula gives for [0.1, 1] (alpha ~1.27, beta ~2.31) */
} sci_solver_params;

/* ---- context ----------------------------------------------------------- */

/* Create a context bound to HIP device `device` (it becomes current on the
 * calling thread). *out receives the handle. */
int sci_create(sci_ctx **out, int device);
/* Free the context's scratch and graphs (synchronises the device first). NULL is a no-op. */
void sci_destroy(sci_ctx *ctx);
/* Static text for a status code. */
const char *sci_status_string(int status);
/* Text of the last failure recorded in the context (empty if none). */
const char *sci_last_error(const sci_ctx *ctx);

/* ---- sensing operator, Eq. (3)-(4) ------------------------------------- */

/* Y_ij = sum_k C_kij X_kij. C, X: video; Y: image (output). The noise term G
 * of Eq. (3) is not added. */
int sci_forward(sci_ctx *ctx, sci_dims d, const float *C, const float *X, float *Y, hipStream_t stream);

/* Transpose of Phi = [D_1 ... D_B] (Eq. (2)): X_kij = C_kij Y_ij. C: video;
 * Y: image; X: video (output). */
int sci_adjoint(sci_ctx *ctx, sci_dims d, const float *C, const float *Y, float *X, hipStream_t stream);

/* ---- TV denoiser (Sec. 2.3, Algorithm 1 FGP/Cham boxes) ------------------ */

/* Theta_out = TVdenoise(X_in) with the dual started from dual_init (NULL =
 * zero). dual_init / dual_out are dual-shaped in p->dual_dtype; dual_out
 * (nullable) receives the final projected dual p^(N); Theta_out is
 * X_in - lambda D^T p^(N). rel_gap_out (nullable, HOST pointer) receives
 * the relative duality gap lambda (TV(theta) - <D theta, p>) / P(theta)
 * computed in FP64; iters_out (nullable, HOST) the iterations run.
 * Returns SCI_NOT_CONVERGED when gap_tol > 0 was not met at n_inner_max,
 * or at the first check whose gap or primal value is not finite (a NaN or
 * infinity in dual_init or X_in): a non-finite gap never meets a tolerance,
 * the loop stops there and *rel_gap_out is NaN. */
int sci_tv_denoise(sci_ctx *ctx, sci_dims d, const sci_tv_params *p, const float *X_in, float *Theta_out,
                   const void *dual_init, void *dual_out, double *rel_gap_out, int32_t *iters_out,
                   hipStream_t stream);

/* ---- outer frameworks ---------------------------------------------------- */

/* GAP (Eq. (21)-(22), Algorithm 1): theta^(0) = Phi^T Y (or X_init);
 *   x^(t+1) = theta^(t) + Phi^T (Phi Phi^T)^+ (Y - Phi theta^(t)),
 *   theta^(t+1) = TVdenoise(x^(t+1)),
 * for exactly outer_iters iterations. (Phi Phi^T)^+ is 1/sum_k C_k^2 where
 * that sum is positive and 0 elsewhere. Y: image; C: video; X_out: video
 * receiving x^(T) (theta^(0) if T = 0); Theta_out (nullable): theta^(T);
 * X_init (nullable): theta^(0). */
int sci_gap_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
               float *X_out, float *Theta_out, const float *X_init, hipStream_t stream);

/* sci_gap_tv for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, and harnesses that forbid
 * hipMalloc. It calls no hipMalloc, hipFree or other allocating routine and
 * creates no event; its scratch (the 1 / S image, the packed masks and their
 * flag, about 32 MiB) is a fixed device array that the library holds on every
 * GPU it runs on until the process ends, so nx * ny <= 4194304
 * (SCI_ERR_INVALID_ARG beyond). Same arguments and results as sci_gap_tv with
 * the same parameters and tile_passes = 1, except: Theta_out is required (it
 * holds theta between iterations); use_graph and warm_dual must be 0
 * (SCI_ERR_UNSUPPORTED); every denoiser call runs as one cold on-chip pass
 * that stores no dual, so n_inner <= 10 (VTV: 10 / 10 / 7 / 4 for
 * B <= 8 / 16 / 24 / 32; SCI_ERR_UNSUPPORTED beyond), schedule and
 * tile_passes are ignored and dual_dtype does not change the result. Every
 * part of the scratch is written before it is read in each call. All calls on
 * one GPU share its array: calls that overlap in time on one GPU (different
 * streams, host threads or contexts) race and must be ordered by the caller. */
int sci_gap_tv_noalloc(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
                       float *X_out, float *Theta_out, const float *X_init, hipStream_t stream);

/* ADMM (Eq. (24)-(26)): theta^(0) = Phi^T Y (or X_init), u^(0) = 0;
 *   x^(t+1) = v + Phi^T (Phi Phi^T + rho I)^{-1} (Y - Phi v), v = theta^(t) - u^(t)
 *   theta^(t+1) = TVdenoise(u^(t) + x^(t+1))   (weight lambda)
 *   u^(t+1) = u^(t) + x^(t+1) - theta^(t+1).
 * Arguments as sci_gap_tv; rho from p->rho (rho = 0 reduces to GAP). */
int sci_admm_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
                float *X_out, float *Theta_out, const float *X_init, hipStream_t stream);

/* FISTA (Sec. 2.2) on 1/2 ||y - Phi x||^2 + lambda TV(x): with L = L(f) =
 * max_ij sum_k C_kij^2 (the largest eigenvalue of Phi^T Phi),
 *   theta^(1) = x^(0) = Phi^T y (or X_init), tau^(1) = 1,
 *   z = theta^(t) + (1/L) Phi^T (y - Phi theta^(t)),
 *   x^(t) = TVdenoise(z) with weight lambda / L (p->tv otherwise),
 *   theta^(t+1) = x^(t) + (tau^(t) - 1) / tau^(t+1) (x^(t) - x^(t-1)).
 * X_out = x^(T); Theta_out (nullable) = theta^(T+1). p->warm_dual = 1 starts
 * each prox call from the previous call's final dual. Runs eagerly (L is read
 * back, which synchronises `stream` once): p->use_graph must be 0.
 * SCI_ERR_INVALID_ARG when every mask entry is 0. */
int sci_fista_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
                 float *Theta_out, const float *X_init, hipStream_t stream);

/* TwIST (Sec. 2.2) on the same objective:
 *   x^(0) = Phi^T y (or X_init); z = x^(t) + (1/L) Phi^T (y - Phi x^(t));
 *   theta^(t) = TVdenoise(z) with weight lambda / L;
 *   x^(1) = theta^(0); x^(t+1) = (1 - alpha) x^(t-1) + (alpha - beta) x^(t) + beta theta^(t).
 * alpha, beta from p->twist_alpha / twist_beta (0 < alpha < 2, beta > 0).
 * X_out = x^(T); Theta_out (nullable) = theta^(T-1) (x^(0) when T = 0).
 * Same restrictions as sci_fista_tv. */
int sci_twist_tv(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C, float *X_out,
                 float *Theta_out, const float *X_init, hipStream_t stream);

/* ---- batched solve --------------------------------------------------------- */

/* One measurement of a batch: sizes, inputs and outputs as for sci_gap_tv. */
typedef struct {
    sci_dims d;
    const float *Y;          /* image [nx][ny] */
    const float *C;          /* masks, video [B][nx][ny] */
    float *X_out;            /* video: x^(T) */
    float *Theta_out;        /* video: theta^(T) (nullable) */
    int32_t outer_iters;     /* > 0: this problem's MaxIter; 0: the batch's p->outer_iters */
} sci_problem;

/* GAP (Eq. (21)-(22)) for n independent measurements of different sizes in
 * one go: each outer iteration is one projection launch and one fused
 * denoise launch that cover every problem still iterating (VTV, Eq. (31)-(32):
 * one row-pipelined denoise pass per such problem), and with p->use_graph the
 * whole loop is one HIP graph launch. Results are bit-identical to
 * sci_gap_tv on each problem with the fused schedule.
 * Requirements: ATV, ITV2D or VTV, lambda > 0, 1 <= n_inner <= 10 (VTV: at
 * most 10 / 8 / 7 / 4 for B <= 8 / 16 / 24 / 32 frames, the longest single
 * pass sci_gap_tv runs unsplit, for every problem), cold start
 * (warm_dual = 0), B <= 32 per problem; dual_dtype and schedule are
 * ignored (the dual never leaves the chip); otherwise SCI_ERR_UNSUPPORTED.
 * Outputs of different problems must not overlap. The tile shape (ATV,
 * ITV2D) is p->tv.tile_shape, else the one sci_autotune_batched chose for
 * this batch, else the default. */
int sci_gap_tv_batched(sci_ctx *ctx, int32_t n, const sci_problem *probs, const sci_solver_params *p,
                       hipStream_t stream);

/* Time the batched denoise launch of this batch with every tile shape and
 * remember the fastest for later sci_gap_tv_batched calls on a batch of the
 * same sizes, TV kind and n_inner. Uses the problems' X_out / Theta_out as
 * scratch. best_shape_out (nullable, HOST): 1-based winner; times_ms_out
 * (nullable, HOST array of sci_tile_shape_count() doubles): mean time of one
 * batched denoise launch per shape. Synchronises `stream`. VTV batches have
 * no tile shape: SCI_ERR_UNSUPPORTED. */
int sci_autotune_batched(sci_ctx *ctx, int32_t n, const sci_problem *probs, const sci_solver_params *p,
                         int32_t *best_shape_out, double *times_ms_out, hipStream_t stream);

/* ---- learned warm start of the TV denoiser ---------------------------------- */

/* A small convolutional network that predicts the denoiser's dual field, so
 * that FGP can start near its solution. Architecture: 4 layers of 3x3x3
 * "same" convolutions over (frame, row, column), c_in -> 16 -> 16 -> 16 ->
 * c_out channels, bias, ReLU after layers 1-3; bf16 weights and activations
 * with fp32 accumulation (MFMA), fp32 master weights and Adam moments.
 * c_in = 1: the input is the denoiser input x and the output (c_out = 2) is
 * the dual (p_h, p_v). c_in = 3: the input is x and a base dual P_base (in
 * the gap-controlled solver: the previous outer iteration's final dual), and
 * the prediction is P_base + output. The paper has no such network; it
 * serves the gap-controlled solver below. One network may be used from one
 * stream at a time. */
typedef struct sci_wsnet sci_wsnet;

int sci_wsnet_create(sci_ctx *ctx, int32_t c_in, int32_t c_out, sci_wsnet **out); /* weights start at 0 */
void sci_wsnet_destroy(sci_wsnet *net);

/* Parameters are exchanged as fp32 in a padded layout: per layer l = 0..3,
 * 28 * 16 * 16 floats [slot][out][in]; slots 0..26 are the taps
 * t = 9 (dk+1) + 3 (di+1) + (dj+1) of offset (dk, di, dj) along
 * (frame, row, column), slot 27 holds the bias in input column 0. Entries
 * outside a layer's channels are ignored (read back as 0). */
int64_t sci_wsnet_param_count(void);
int sci_wsnet_set_params(sci_ctx *ctx, sci_wsnet *net, const float *host, int64_t count); /* resets Adam */
int sci_wsnet_get_params(sci_ctx *ctx, sci_wsnet *net, float *host, int64_t count);

/* Network output for input X (video) and, when c_in = 3, P_base (dual
 * [2][B][nx][ny] fp32; NULL = zero; ignored when c_in = 1): Y_out (nullable)
 * [c_out][B][nx][ny] fp32 raw output, dual_out (nullable) [2][B][nx][ny]
 * fp32 = (P_base +) output projected onto the dual ball of TV kind tv with
 * the entries that carry no difference set to 0 (c_out = 2). */
int sci_wsnet_forward(sci_ctx *ctx, sci_wsnet *net, sci_dims d, const float *X, const float *P_base, float *Y_out,
                      int32_t tv, float *dual_out, hipStream_t stream);

/* Training loss of a network (default SCI_WSNET_LOSS_DUAL):
 *   SCI_WSNET_LOSS_DUAL : 1/(c_out V) sum (r)^2 over the c_out channels,
 *   SCI_WSNET_LOSS_THETA: 1/V sum (D^T r)^2 over the voxels (c_out = 2),
 * with r = (P_base +) y - target and, for THETA, r held at 0 on the dual
 * entries that carry no difference. The denoiser's primal theta = x -
 * lambda D^T p and its duality gap depend on the dual only through D^T p
 * (Sec. 2.3, FGP), and the optimal dual is not unique; THETA ignores the
 * null-space components of D^T in which converged duals differ. Unknown
 * kind, or THETA with c_out != 2: SCI_ERR_INVALID_ARG. */
typedef enum { SCI_WSNET_LOSS_DUAL = 0, SCI_WSNET_LOSS_THETA = 1 } sci_wsnet_loss;
int sci_wsnet_set_loss(sci_ctx *ctx, sci_wsnet *net, int32_t kind);

/* The network's loss (sci_wsnet_set_loss) for target [c_out][B][nx][ny]
 * fp32 and its gradient for every parameter (HOST, padded layout), without
 * an update. Synchronises `stream`. */
int sci_wsnet_grads(sci_ctx *ctx, sci_wsnet *net, sci_dims d, const float *X, const float *P_base, const float *target,
                    float *grad_host, double *loss_host, hipStream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on that
 * loss; loss_host (nullable) receives the loss before the step (then the call
 * synchronises `stream`). */
int sci_wsnet_train_step(sci_ctx *ctx, sci_wsnet *net, sci_dims d, const float *X, const float *P_base,
                         const float *target, float lr, double *loss_host, hipStream_t stream);

/* GAP (Eq. (21)-(22)) whose denoiser runs until the relative duality gap
 * <= p->tv.gap_tol (checked every p->tv.gap_check_every iterations, at most
 * p->tv.n_inner_max per outer iteration), each call starting from: the
 * network's projected prediction (net non-null; a network with c_in = 3 gets
 * the previous outer iteration's final dual as P_base and is not used in the
 * first outer iteration, which has none; with p->warm_dual = 1 as well, the
 * call starts from whichever of the prediction and the previous final dual
 * has the smaller relative duality gap, a non-finite gap losing; when a
 * call that started from the prediction does not reach the tolerance, or
 * meets a non-finite gap, it is repeated from a zero dual), else the
 * previous outer iteration's final dual (p->warm_dual = 1), else zero.
 * A call started from the previous final dual is not repeated (as without
 * a network).
 * inner_iters_out / fallbacks_out / net_starts_out (nullable, HOST): total
 * inner iterations (fallbacks included), the number of cold-start
 * fallbacks, and the number of calls that started from the prediction.
 * float32 duals; synchronises `stream` at every gap check. */
int sci_gap_tv_adaptive(sci_ctx *ctx, sci_dims d, const sci_solver_params *p, const float *Y, const float *C,
                        float *X_out, float *Theta_out, const float *X_init, sci_wsnet *net, int32_t *inner_iters_out,
                        int32_t *fallbacks_out, int32_t *net_starts_out, hipStream_t stream);

/* ---- tile-shape autotuning of the fused schedule -------------------------- */

/* Number of shapes of the fused denoiser (tiled, then row-pipelined). */
int sci_tile_shape_count(void);

/* Shape k (1-based, as in sci_tv_params.tile_shape). Tiled shape: a
 * workgroup covers 64 * cols_per_lane columns x (rows_per_wave *
 * waves_per_group) rows of one frame, halo included, and keeps the whole tile
 * on chip for a pass. Row-pipelined shape (sci_tile_shape_pipelined): one
 * wavefront (waves_per_group = 1) walks a segment of rows_per_wave rows of a
 * strip of 64 * cols_per_lane columns, halo columns included, from top to
 * bottom, every iteration of the pass one row behind the previous one
 * (temporal wavefront blocking; no rows are recomputed apart from the
 * pipeline fill of about 2 n rows per segment). Row-pipelined shapes run
 * float32 dual storage; with 16-bit storage they serve cold passes that
 * neither read nor return the dual (the storage is then never touched), and
 * any other 16-bit pass runs the default shape. Any output pointer may be
 * NULL. */
int sci_tile_shape_info(int32_t shape, int32_t *rows_per_wave, int32_t *waves_per_group, int32_t *cols_per_lane);

/* 1 if shape k (1-based) is row-pipelined, 0 if tiled, SCI_ERR_INVALID_ARG
 * for a shape out of range. */
int sci_tile_shape_pipelined(int32_t shape);

/* Time the fused denoiser (p->tv, p->lambda, p->n_inner, p->dual_dtype) on
 * input X (video, device) for every tile shape and for 3 pass counts (the
 * fewest passes of at most 10 iterations, one more, two more), and remember
 * the fastest pair in the context for later calls with the same TV kind,
 * dual dtype, sizes and n_inner whose tile_shape / tile_passes are 0. With
 * p->schedule == SCI_SCHED_STREAM the one-iteration-per-pass configuration
 * is tuned instead (tile shape only; the other pass-count entries are NaN).
 * best_shape_out / best_passes_out (nullable, HOST) receive the winner;
 * times_ms_out (nullable, HOST array of 3 * sci_tile_shape_count() doubles,
 * [shape][pass-count candidate]) the mean time per denoiser call, NaN where a
 * candidate was skipped. Synchronises `stream`. ATV and ITV2D only
 * (SCI_ERR_UNSUPPORTED for VTV). */
int sci_autotune(sci_ctx *ctx, sci_dims d, const sci_tv_params *p, const float *X, int32_t *best_shape_out,
                 int32_t *best_passes_out, double *times_ms_out, hipStream_t stream);

/* ---- FP64 reductions on the GPU (results to HOST pointers) ---------------- */

/* 10 log10(peak^2 / MSE), MSE over `count` floats of a against ref. */
int sci_psnr(sci_ctx *ctx, int64_t count, const float *a, const float *ref, double peak, double *out_host,
             hipStream_t stream);

/* ||Y - Phi X||^2 (Eq. (6) data term times 2). */
int sci_residual_sq(sci_ctx *ctx, sci_dims d, const float *C, const float *X, const float *Y, double *out_host,
                    hipStream_t stream);

/* Duality gap of the denoising problem at the dual p (dual-shaped, storage
 * type dual_dtype): gap = lambda (TV(theta) - <D theta, p>) and primal
 * P(theta) = 1/2 ||theta - x||^2 + lambda TV(theta) with
 * theta = x - lambda D^T p, all in FP64, summed in a fixed order
 * (repeated calls return identical values). Either host output may be
 * NULL. VTV with B > 48: SCI_ERR_UNSUPPORTED (as for the VTV denoiser). */
int sci_dual_gap(sci_ctx *ctx, sci_dims d, int32_t tv, int32_t dual_dtype, float lambda, const float *X,
                 const void *p, double *gap_host, double *primal_host, hipStream_t stream);

/* ---- kernel timing (the library's own tracing) -------------------------- */

/* enable != 0: from now on record a HIP event pair on the launch stream
 * around every kernel the solver entry points launch outside graph capture
 * (earlier records are cleared); enable == 0 stops recording. */
int sci_profile_enable(sci_ctx *ctx, int enable);

/* Number of recorded launches and their summed duration (milliseconds, from
 * hipEventElapsedTime) for one kernel family: "fgp_stream" (one inner
 * iteration over HBM), "fgp_fused" (all inner iterations on chip),
 * "tv_theta" (theta = x - lambda D^T p), "project" (GAP / ADMM projection),
 * "setup" (weights, Phi^T y, copies). Synchronises on the recorded events.
 * Unknown family: SCI_ERR_INVALID_ARG. */
int sci_profile_read(sci_ctx *ctx, const char *family, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SCITV_H */
