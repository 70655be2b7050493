/*
 * FP64 CPU oracle for TV-regularised reconstruction of snapshot video
 * compressive imaging (X. Yuan, "Various Total Variation for Snapshot Video
 * Compressive Imaging", arXiv:2005.08028).
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow reference that the HIP
 * library is checked against. Only the test suite, the package smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does. It shares no code, header, table or constant generator with the HIP
 * library.
 *
 * Everything is double precision, scalar loops, no blocking or fusion; the
 * only parallelism is an OpenMP split of element-wise loops (each output
 * element is computed by exactly the same expression whatever the thread
 * count). Reductions run serially in a fixed order.
 *
 * Layout (row-major, column index fastest):
 *   video   [B][nx][ny]   frame k, row i, column j           (Eq. (3), (5))
 *   image   [nx][ny]
 *   dual    [2][B][nx][ny] channel 0 = horizontal (h), 1 = vertical (v)
 *
 * Readings of the paper that this file takes (each is listed, with its
 * reason, in the design notes of the repository):
 *   - D_h differences along columns j, D_v along rows i (Eq. (7)): forward
 *     differences, no wrap-around. The dual field keeps full size; the
 *     entries with no difference (j = ny-1 for h, i = nx-1 for v) are zero
 *     in D(theta) and are ignored by D^T.
 *   - ITV2D / ITV3D are taken per pixel (isotropic at every voxel, resp. a
 *     norm over all 2B values at a pixel) as the dual projections
 *     Eq. (29)-(32) define them.
 *   - FGP: nu^(0) = 1, w^(0) = p^(0) = 0 (or a caller warm start), exactly
 *     N inner iterations, output theta = x - lambda D^T p^(N) from the last
 *     projected dual (a flag selects the literal theta^(N) built from the
 *     extrapolated w^(N-1)).
 *   - Chambolle's projected gradient is FGP without extrapolation; its step
 *     moves the dual along +D(x - lambda D^T w) (the sign that decreases the
 *     denoising objective).
 *   - (Phi Phi^T)^{-1} is the Moore-Penrose inverse of the diagonal
 *     S = sum_k C_k^2 (zero where S = 0).
 *   - ADMM denoises u + x with weight lambda; rho only enters the x-update.
 *   - lambda = 0 or N = 0 returns the denoiser input unchanged.
 *
 * Parity status: every function below is pinned by the CPU tests (adjoint
 * identities, dense-matrix formulations built from Eq. (2) and Eq. (7),
 * closed-form TV values and prox solutions, an independent bound-constrained
 * dual solve, fixed points and normal equations; ADMM, FISTA and TwIST by
 * hand-worked three-iteration examples, and ADMM's limit by an independent
 * constrained solve of the penalised least-squares problem it minimises).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ATV 0
#define ORC_ITV2D 1
#define ORC_VTV 2

#define IDX(k, i, j) (((size_t)(k) * (size_t)nx + (size_t)(i)) * (size_t)ny + (size_t)(j))

/* Threads of the element-wise loops for later calls from this thread (the
 * results do not depend on it); used to time the oracle at one thread and at
 * all cores. Returns the count now in effect. */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Sensing operator, Eq. (2)-(4): Y = sum_k C_k .* X_k, and its transpose.  */
/* ------------------------------------------------------------------------ */

/* Y_ij = sum_k C_kij X_kij  (Eq. (4), noise excluded). */
void orc_forward(int B, int nx, int ny, const double *C, const double *X, double *Y)
{
#pragma omp parallel for
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double acc = 0.0;
            for (int k = 0; k < B; ++k)
                acc += C[IDX(k, i, j)] * X[IDX(k, i, j)];
            Y[(size_t)i * ny + j] = acc;
        }
}

/* Phi^T: X_kij = C_kij Y_ij (transpose of the block row [D_1 ... D_B], Eq. (2)). */
void orc_adjoint(int B, int nx, int ny, const double *C, const double *Y, double *X)
{
#pragma omp parallel for
    for (int k = 0; k < B; ++k)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j)
                X[IDX(k, i, j)] = C[IDX(k, i, j)] * Y[(size_t)i * ny + j];
}

/* diag(Phi Phi^T) = sum_k C_k^2, and the element-wise inverse used by the
 * projection: 1 / (S + rho) where that is positive, 0 elsewhere. */
void orc_weights(int B, int nx, int ny, const double *C, double rho, double *Sinv)
{
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double s = 0.0;
            for (int k = 0; k < B; ++k)
                s += C[IDX(k, i, j)] * C[IDX(k, i, j)];
            s += rho;
            Sinv[(size_t)i * ny + j] = (s > 0.0) ? 1.0 / s : 0.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Finite differences, Eq. (7).                                             */
/* ------------------------------------------------------------------------ */

/* D theta: h = theta(i, j+1) - theta(i, j), v = theta(i+1, j) - theta(i, j);
 * zero where the neighbour does not exist. */
void orc_grad(int B, int nx, int ny, const double *th, double *gh, double *gv)
{
#pragma omp parallel for
    for (int k = 0; k < B; ++k)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                size_t c = IDX(k, i, j);
                gh[c] = (j + 1 < ny) ? th[IDX(k, i, j + 1)] - th[c] : 0.0;
                gv[c] = (i + 1 < nx) ? th[IDX(k, i + 1, j)] - th[c] : 0.0;
            }
}

/* D^T p, the exact adjoint of orc_grad: entries of p with no difference
 * behind them (j = ny-1 in h, i = nx-1 in v) do not contribute. */
void orc_grad_adj(int B, int nx, int ny, const double *ph, const double *pv, double *out)
{
#pragma omp parallel for
    for (int k = 0; k < B; ++k)
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                double a = 0.0;
                if (j >= 1) a += ph[IDX(k, i, j - 1)];       /* from difference (j-1, j) */
                if (j + 1 < ny) a -= ph[IDX(k, i, j)];       /* from difference (j, j+1) */
                if (i >= 1) a += pv[IDX(k, i - 1, j)];
                if (i + 1 < nx) a -= pv[IDX(k, i, j)];
                out[IDX(k, i, j)] = a;
            }
}

/* ------------------------------------------------------------------------ */
/* TV values, Eq. (8)-(10) (per-pixel reading of the isotropic forms).      */
/* ------------------------------------------------------------------------ */

double orc_tv_value(int kind, int B, int nx, int ny, const double *th)
{
    size_t V = (size_t)B * nx * ny;
    double *gh = (double *)malloc(V * sizeof(double));
    double *gv = (double *)malloc(V * sizeof(double));
    orc_grad(B, nx, ny, th, gh, gv);
    double tv = 0.0;
    if (kind == ORC_ATV) {
        for (size_t c = 0; c < V; ++c) tv += fabs(gh[c]) + fabs(gv[c]);
    } else if (kind == ORC_ITV2D) {
        for (size_t c = 0; c < V; ++c) tv += sqrt(gh[c] * gh[c] + gv[c] * gv[c]);
    } else {
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                double s = 0.0;
                for (int k = 0; k < B; ++k) {
                    size_t c = IDX(k, i, j);
                    s += gh[c] * gh[c] + gv[c] * gv[c];
                }
                tv += sqrt(s);
            }
    }
    free(gh);
    free(gv);
    return tv;
}

/* ------------------------------------------------------------------------ */
/* Dual projection onto the unit ball of the TV's dual norm.                */
/*   ATV   : each of q_h, q_v divided by max(1, |.|)     (Algorithm 1, FGP) */
/*   ITV2D : (q_h, q_v) per voxel divided by max(1, ||.||)  (Eq. (29)-(30)) */
/*   VTV   : all 2B values of a pixel divided by max(1, ||.||) (Eq. (31)-(32)) */
/* ------------------------------------------------------------------------ */

void orc_project_dual(int kind, int B, int nx, int ny, double *qh, double *qv)
{
    size_t V = (size_t)B * nx * ny;
    if (kind == ORC_ATV) {
#pragma omp parallel for
        for (long c = 0; c < (long)V; ++c) {
            qh[c] = qh[c] / fmax(1.0, fabs(qh[c]));
            qv[c] = qv[c] / fmax(1.0, fabs(qv[c]));
        }
    } else if (kind == ORC_ITV2D) {
#pragma omp parallel for
        for (long c = 0; c < (long)V; ++c) {
            double d = fmax(1.0, sqrt(qh[c] * qh[c] + qv[c] * qv[c]));
            qh[c] = qh[c] / d;
            qv[c] = qv[c] / d;
        }
    } else {
#pragma omp parallel for
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                double s = 0.0;
                for (int k = 0; k < B; ++k) {
                    size_t c = IDX(k, i, j);
                    s += qh[c] * qh[c] + qv[c] * qv[c];
                }
                double d = fmax(1.0, sqrt(s));
                for (int k = 0; k < B; ++k) {
                    size_t c = IDX(k, i, j);
                    qh[c] = qh[c] / d;
                    qv[c] = qv[c] / d;
                }
            }
    }
}

/* Dual entries that carry no difference are kept at zero. */
static void zero_padding(int B, int nx, int ny, double *ph, double *pv)
{
    for (int k = 0; k < B; ++k) {
        for (int i = 0; i < nx; ++i) ph[IDX(k, i, ny - 1)] = 0.0;
        for (int j = 0; j < ny; ++j) pv[IDX(k, nx - 1, j)] = 0.0;
    }
}

/* FGP momentum: nu^(s+1) = (1 + sqrt(1 + 4 nu^(s)^2)) / 2 with nu^(0) = 1,
 * beta_s = (nu^(s) - 1) / nu^(s+1)  (Algorithm 1, FGP box). */
void orc_fgp_beta(int n, double *beta)
{
    double nu = 1.0;
    for (int s = 0; s < n; ++s) {
        double nu1 = (1.0 + sqrt(1.0 + 4.0 * nu * nu)) / 2.0;
        beta[s] = (nu - 1.0) / nu1;
        nu = nu1;
    }
}

/* ------------------------------------------------------------------------ */
/* TV denoiser: theta = argmin 1/2 ||theta - x||^2 + lambda TV(theta),      */
/* by Beck-Teboulle's fast gradient projection on the dual (accel = 1) or   */
/* Chambolle's projected gradient (accel = 0), step 1/(8 lambda).           */
/* Algorithm 1 (ATV-FGP and ATV-Cham boxes), Eq. (27)-(32) for ITV2D/ITV3D. */
/*                                                                          */
/* p_init: optional warm-start dual [2][B][nx][ny] (NULL = zero).           */
/* chambolle04: use the semi-implicit denominator 1 + |z|/(8 lambda) of     */
/*   Chambolle (2004) in place of max(1, |q|) (Sec. 2.3, ATV-FGP note),     */
/*   with q measured per the TV kind.                                       */
/* literal_out: return theta^(N) = x - lambda D^T w^(N-1) instead of        */
/*   x - lambda D^T p^(N).                                                  */
/* theta_out: [B][nx][ny]; ph_out / pv_out: optional final dual.            */
/* ------------------------------------------------------------------------ */
int orc_tv_denoise(int kind, int B, int nx, int ny, double lambda, int n_iter, int accel,
                   int chambolle04, int literal_out, const double *x, const double *p_init,
                   double *theta_out, double *ph_out, double *pv_out)
{
    size_t V = (size_t)B * nx * ny;
    if (lambda == 0.0 || n_iter == 0) {
        memcpy(theta_out, x, V * sizeof(double));
        if (ph_out) {
            if (p_init) { memmove(ph_out, p_init, V * sizeof(double)); memmove(pv_out, p_init + V, V * sizeof(double)); }
            else { memset(ph_out, 0, V * sizeof(double)); memset(pv_out, 0, V * sizeof(double)); }
        }
        return 0;
    }
    double *ph = (double *)calloc(V, sizeof(double)), *pv = (double *)calloc(V, sizeof(double));
    double *wh = (double *)calloc(V, sizeof(double)), *wv = (double *)calloc(V, sizeof(double));
    double *qh = (double *)malloc(V * sizeof(double)), *qv = (double *)malloc(V * sizeof(double));
    double *th = (double *)malloc(V * sizeof(double)), *dt = (double *)malloc(V * sizeof(double));
    if (p_init) {
        memcpy(ph, p_init, V * sizeof(double));
        memcpy(pv, p_init + V, V * sizeof(double));
        zero_padding(B, nx, ny, ph, pv);
    }
    memcpy(wh, ph, V * sizeof(double));
    memcpy(wv, pv, V * sizeof(double));
    const double step = 1.0 / (8.0 * lambda);
    double nu = 1.0;
    for (int s = 0; s < n_iter; ++s) {
        /* theta^(s+1) = x - lambda D^T w^(s) */
        orc_grad_adj(B, nx, ny, wh, wv, dt);
        for (size_t c = 0; c < V; ++c) th[c] = x[c] - lambda * dt[c];
        /* z^(s+1) = D theta^(s+1);  q = w^(s) + z / (8 lambda) */
        orc_grad(B, nx, ny, th, qh, qv);
        if (!chambolle04) {
            for (size_t c = 0; c < V; ++c) { qh[c] = wh[c] + step * qh[c]; qv[c] = wv[c] + step * qv[c]; }
            orc_project_dual(kind, B, nx, ny, qh, qv);    /* p^(s+1) = P_K(q) */
        } else {
            /* p = (w + dt z) / (1 + dt |z|), |z| taken per the TV kind */
            double *den = dt; /* reuse */
            if (kind == ORC_ATV) {
                for (size_t c = 0; c < V; ++c) {
                    double zh = qh[c], zv = qv[c];
                    qh[c] = (wh[c] + step * zh) / (1.0 + step * fabs(zh));
                    qv[c] = (wv[c] + step * zv) / (1.0 + step * fabs(zv));
                }
            } else if (kind == ORC_ITV2D) {
                for (size_t c = 0; c < V; ++c) {
                    double d = 1.0 + step * sqrt(qh[c] * qh[c] + qv[c] * qv[c]);
                    qh[c] = (wh[c] + step * qh[c]) / d;
                    qv[c] = (wv[c] + step * qv[c]) / d;
                }
            } else {
                for (int i = 0; i < nx; ++i)
                    for (int j = 0; j < ny; ++j) {
                        double sq = 0.0;
                        for (int k = 0; k < B; ++k) {
                            size_t c = IDX(k, i, j);
                            sq += qh[c] * qh[c] + qv[c] * qv[c];
                        }
                        den[(size_t)i * ny + j] = 1.0 + step * sqrt(sq);
                    }
                for (int k = 0; k < B; ++k)
                    for (int i = 0; i < nx; ++i)
                        for (int j = 0; j < ny; ++j) {
                            size_t c = IDX(k, i, j);
                            double d = den[(size_t)i * ny + j];
                            qh[c] = (wh[c] + step * qh[c]) / d;
                            qv[c] = (wv[c] + step * qv[c]) / d;
                        }
            }
        }
        zero_padding(B, nx, ny, qh, qv);
        /* nu^(s+1), and w^(s+1) = p^(s+1) + (nu^(s) - 1)/nu^(s+1) (p^(s+1) - p^(s)) */
        double nu1 = (1.0 + sqrt(1.0 + 4.0 * nu * nu)) / 2.0;
        double beta = accel ? (nu - 1.0) / nu1 : 0.0;
        if (literal_out && s == n_iter - 1) break; /* theta^(N) already in th */
        for (size_t c = 0; c < V; ++c) {
            wh[c] = qh[c] + beta * (qh[c] - ph[c]);
            wv[c] = qv[c] + beta * (qv[c] - pv[c]);
            ph[c] = qh[c];
            pv[c] = qv[c];
        }
        nu = nu1;
    }
    if (literal_out) {
        memcpy(theta_out, th, V * sizeof(double));
        /* the final projected dual is in q */
        memcpy(ph, qh, V * sizeof(double));
        memcpy(pv, qv, V * sizeof(double));
    } else {
        orc_grad_adj(B, nx, ny, ph, pv, dt);
        for (size_t c = 0; c < V; ++c) theta_out[c] = x[c] - lambda * dt[c];
    }
    if (ph_out) {
        memcpy(ph_out, ph, V * sizeof(double));
        memcpy(pv_out, pv, V * sizeof(double));
    }
    free(ph); free(pv); free(wh); free(wv); free(qh); free(qv); free(th); free(dt);
    return 0;
}

/* ATV-Clip (Sec. 2.3; Algorithm 1, Clip box): iterative clipping with one
 * dual per difference direction. Threshold T = 2 lambda (as printed), step
 * 1/alpha; for s = 0 .. n_iter-1:
 *   theta_h = x - D_h^T w_h,   theta_v = x - D_v^T w_v,
 *   w_h <- clip(w_h + D_h theta_h / alpha, T),   w_v <- clip(w_v + D_v theta_v / alpha, T),
 * output theta = theta_h + theta_v - x = x - D_h^T w_h - D_v^T w_v, taken with
 * the final duals (the convention used for every denoiser here). Each
 * direction is projected gradient on the dual of
 * 1/2 ||theta - x||^2 + T ||D_d theta||_1, convergent for alpha > 2 since
 * ||D_d D_d^T|| < 4. w_init: optional [2][B][nx][ny] start. */
int orc_clip_denoise(int B, int nx, int ny, double lambda, double alpha, int n_iter, const double *x,
                     const double *w_init, double *theta_out, double *wh_out, double *wv_out)
{
    size_t V = (size_t)B * nx * ny;
    double *wh = (double *)calloc(V, sizeof(double)), *wv = (double *)calloc(V, sizeof(double));
    double *zero = (double *)calloc(V, sizeof(double));
    double *th = (double *)malloc(V * sizeof(double)), *tv = (double *)malloc(V * sizeof(double));
    double *gh = (double *)malloc(V * sizeof(double)), *gv = (double *)malloc(V * sizeof(double));
    double *dt = (double *)malloc(V * sizeof(double));
    if (w_init) {
        memcpy(wh, w_init, V * sizeof(double));
        memcpy(wv, w_init + V, V * sizeof(double));
        zero_padding(B, nx, ny, wh, wv);
    }
    const double T = 2.0 * lambda;
    for (int s = 0; s < n_iter; ++s) {
        orc_grad_adj(B, nx, ny, wh, zero, dt); /* D_h^T w_h */
        for (size_t c = 0; c < V; ++c) th[c] = x[c] - dt[c];
        orc_grad_adj(B, nx, ny, zero, wv, dt); /* D_v^T w_v */
        for (size_t c = 0; c < V; ++c) tv[c] = x[c] - dt[c];
        orc_grad(B, nx, ny, th, gh, dt);       /* D_h theta_h (the v part is unused) */
        orc_grad(B, nx, ny, tv, dt, gv);       /* D_v theta_v */
        for (size_t c = 0; c < V; ++c) {
            double a = wh[c] + gh[c] / alpha, b = wv[c] + gv[c] / alpha;
            wh[c] = a > T ? T : (a < -T ? -T : a);
            wv[c] = b > T ? T : (b < -T ? -T : b);
        }
        zero_padding(B, nx, ny, wh, wv);
    }
    orc_grad_adj(B, nx, ny, wh, wv, dt);
    for (size_t c = 0; c < V; ++c) theta_out[c] = x[c] - dt[c];
    if (wh_out) {
        memcpy(wh_out, wh, V * sizeof(double));
        memcpy(wv_out, wv, V * sizeof(double));
    }
    free(wh); free(wv); free(zero); free(th); free(tv); free(gh); free(gv); free(dt);
    return 0;
}

/* The denoiser of the outer loops: variant 0 = FGP / projected gradient
 * (accel), 1 = with Chambolle's 2004 denominator, 2 = ATV-Clip (step
 * 1/clip_alpha). p (nullable) is the starting dual, p_out [2][V] the final one. */
static void outer_denoise(int kind, int B, int nx, int ny, double lambda, int N, int accel, int variant,
                          double clip_alpha, const double *x, const double *p, double *theta, double *p_out)
{
    size_t V = (size_t)B * nx * ny;
    if (variant == 2) {
        if (lambda == 0.0 || N == 0) {
            memcpy(theta, x, V * sizeof(double));
            if (!p) memset(p_out, 0, 2 * V * sizeof(double));
            else if (p != p_out) memmove(p_out, p, 2 * V * sizeof(double));
            return;
        }
        orc_clip_denoise(B, nx, ny, lambda, clip_alpha, N, x, p, theta, p_out, p_out + V);
    } else {
        orc_tv_denoise(kind, B, nx, ny, lambda, N, accel, variant == 1, 0, x, p, theta, p_out, p_out + V);
    }
}

/* Duality gap of the denoising problem for a feasible dual p, with
 * theta = x - lambda D^T p:
 *   primal  P(theta) = 1/2 ||theta - x||^2 + lambda TV(theta)
 *   dual    Q(p)     = 1/2 ||x||^2 - 1/2 ||x - lambda D^T p||^2
 *   gap     P - Q    = lambda (TV(theta) - <D theta, p>)   (expanded form,
 *                      no cancellation of the two large terms).
 * Returns the gap; *primal_out (optional) receives P(theta). */
double orc_dual_gap(int kind, int B, int nx, int ny, double lambda, const double *x,
                    const double *p, double *primal_out)
{
    size_t V = (size_t)B * nx * ny;
    const double *ph = p, *pv = p + V;
    double *th = (double *)malloc(V * sizeof(double));
    double *gh = (double *)malloc(V * sizeof(double));
    double *gv = (double *)malloc(V * sizeof(double));
    orc_grad_adj(B, nx, ny, ph, pv, th);
    for (size_t c = 0; c < V; ++c) th[c] = x[c] - lambda * th[c];
    double tv = orc_tv_value(kind, B, nx, ny, th);
    orc_grad(B, nx, ny, th, gh, gv);
    double inner = 0.0, fid = 0.0;
    for (size_t c = 0; c < V; ++c) {
        inner += gh[c] * ph[c] + gv[c] * pv[c];
        fid += (th[c] - x[c]) * (th[c] - x[c]);
    }
    if (primal_out) *primal_out = 0.5 * fid + lambda * tv;
    free(th); free(gh); free(gv);
    return lambda * (tv - inner);
}

/* ------------------------------------------------------------------------ */
/* Outer frameworks.                                                        */
/* ------------------------------------------------------------------------ */

/* GAP, Eq. (21)-(22) and Algorithm 1:
 *   theta^(0) = Phi^T y (or x_init)
 *   x^(t+1)     = theta^(t) + Phi^T (Phi Phi^T)^+ (y - Phi theta^(t))
 *   theta^(t+1) = TVdenoise(x^(t+1))
 * for exactly T outer iterations; returns x^(T) and theta^(T).
 * warm: each denoiser call starts from the dual the previous call ended with
 *   (Algorithm 1 initialises p before the outer loop; the first call starts
 *   from zero); otherwise every call starts from zero.
 * variant: 0 = FGP / projected gradient, 1 = Chambolle's 2004 denominator,
 *   2 = ATV-Clip with step 1/clip_alpha (Sec. 2.3, Algorithm 1). */
int orc_gap_tv(int kind, int B, int nx, int ny, double lambda, int T, int N, int accel, int warm, int variant,
               double clip_alpha, const double *Y, const double *C, const double *x_init, double *x_out,
               double *theta_out)
{
    size_t V = (size_t)B * nx * ny, n = (size_t)nx * ny;
    double *Sinv = (double *)malloc(n * sizeof(double));
    double *r = (double *)malloc(n * sizeof(double));
    double *th = (double *)malloc(V * sizeof(double));
    double *x = (double *)malloc(V * sizeof(double));
    double *cr = (double *)malloc(V * sizeof(double));
    double *P = (double *)calloc(2 * V, sizeof(double)); /* carried dual [2][V] */
    orc_weights(B, nx, ny, C, 0.0, Sinv);
    if (x_init) memcpy(th, x_init, V * sizeof(double));
    else orc_adjoint(B, nx, ny, C, Y, th);
    if (T == 0) memcpy(x, th, V * sizeof(double));
    for (int t = 0; t < T; ++t) {
        orc_forward(B, nx, ny, C, th, r);                    /* Phi theta */
        for (size_t c = 0; c < n; ++c) r[c] = (Y[c] - r[c]) * Sinv[c];
        orc_adjoint(B, nx, ny, C, r, cr);                    /* Phi^T (.) */
        for (size_t c = 0; c < V; ++c) x[c] = th[c] + cr[c];
        outer_denoise(kind, B, nx, ny, lambda, N, accel, variant, clip_alpha, x, warm ? P : NULL, th, P);
    }
    memcpy(x_out, x, V * sizeof(double));
    if (theta_out) memcpy(theta_out, th, V * sizeof(double));
    free(Sinv); free(r); free(th); free(x); free(cr); free(P);
    return 0;
}

/* ADMM, Eq. (24)-(26) with theta^(0) = Phi^T y (or x_init), u^(0) = 0:
 *   x^(t+1)     = argmin 1/2||y - Phi x||^2 + rho/2 ||x - theta^(t) + u^(t)||^2
 *               = v + Phi^T (Phi Phi^T + rho I)^{-1} (y - Phi v),  v = theta^(t) - u^(t)
 *     (matrix inversion lemma; Phi Phi^T is diagonal so this is element-wise)
 *   theta^(t+1) = TVdenoise(u^(t) + x^(t+1))  with weight lambda
 *   u^(t+1)     = u^(t) + x^(t+1) - theta^(t+1). */
int orc_admm_tv(int kind, int B, int nx, int ny, double lambda, double rho, int T, int N, int accel, int warm,
                int variant, double clip_alpha, const double *Y, const double *C, const double *x_init,
                double *x_out, double *theta_out)
{
    size_t V = (size_t)B * nx * ny, n = (size_t)nx * ny;
    double *P = (double *)calloc(2 * V, sizeof(double)); /* carried dual [2][V] (warm, as in GAP) */
    double *Sinv = (double *)malloc(n * sizeof(double));
    double *r = (double *)malloc(n * sizeof(double));
    double *th = (double *)malloc(V * sizeof(double));
    double *u = (double *)calloc(V, sizeof(double));
    double *v = (double *)malloc(V * sizeof(double));
    double *x = (double *)malloc(V * sizeof(double));
    double *cr = (double *)malloc(V * sizeof(double));
    orc_weights(B, nx, ny, C, rho, Sinv);
    if (x_init) memcpy(th, x_init, V * sizeof(double));
    else orc_adjoint(B, nx, ny, C, Y, th);
    if (T == 0) memcpy(x, th, V * sizeof(double));
    for (int t = 0; t < T; ++t) {
        for (size_t c = 0; c < V; ++c) v[c] = th[c] - u[c];
        orc_forward(B, nx, ny, C, v, r);
        for (size_t c = 0; c < n; ++c) r[c] = (Y[c] - r[c]) * Sinv[c];
        orc_adjoint(B, nx, ny, C, r, cr);
        for (size_t c = 0; c < V; ++c) x[c] = v[c] + cr[c];
        for (size_t c = 0; c < V; ++c) v[c] = u[c] + x[c];  /* denoiser input */
        outer_denoise(kind, B, nx, ny, lambda, N, accel, variant, clip_alpha, v, warm ? P : NULL, th, P);
        for (size_t c = 0; c < V; ++c) u[c] = u[c] + x[c] - th[c];
    }
    memcpy(x_out, x, V * sizeof(double));
    if (theta_out) memcpy(theta_out, th, V * sizeof(double));
    free(Sinv); free(r); free(th); free(u); free(v); free(x); free(cr); free(P);
    return 0;
}

/* L(f) for f(x) = 1/2 ||y - Phi x||^2: the largest eigenvalue of Phi^T Phi,
 * which equals that of Phi Phi^T = diag(S), S_ij = sum_k C_kij^2 (Sec. 2.2,
 * FISTA; the nonzero spectra of Phi^T Phi and Phi Phi^T coincide). */
double orc_lipschitz(int B, int nx, int ny, const double *C)
{
    double L = 0.0;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            double s = 0.0;
            for (int k = 0; k < B; ++k) {
                const double c = C[IDX(k, i, j)];
                s += c * c;
            }
            if (s > L) L = s;
        }
    return L;
}

/* z = theta + (1/L) Phi^T (y - Phi theta): the gradient step on f. */
static void grad_step(int B, int nx, int ny, const double *C, const double *Y, double invL, const double *th,
                      double *r, double *cr, double *z)
{
    size_t V = (size_t)B * nx * ny, n = (size_t)nx * ny;
    orc_forward(B, nx, ny, C, th, r);
    for (size_t c = 0; c < n; ++c) r[c] = (Y[c] - r[c]) * invL;
    orc_adjoint(B, nx, ny, C, r, cr);
    for (size_t c = 0; c < V; ++c) z[c] = th[c] + cr[c];
}

/* FISTA (Sec. 2.2) for 1/2 ||y - Phi x||^2 + lambda TV(x):
 *   theta^(1) = x^(0) = Phi^T y (or x_init), tau^(1) = 1
 *   z^(t)       = theta^(t) + (1/L) Phi^T (y - Phi theta^(t))
 *   x^(t)       = TVdenoise(z^(t)) with weight lambda / L (the proximal step
 *                 of lambda TV at step 1/L)
 *   tau^(t+1)   = (1 + sqrt(1 + 4 tau^(t)^2)) / 2
 *   theta^(t+1) = x^(t) + (tau^(t) - 1) / tau^(t+1) (x^(t) - x^(t-1))
 * (the printed extrapolation uses x^(t+1) - x^(t), which is not yet known at
 * that point; Beck and Teboulle's method extrapolates along x^(t) - x^(t-1)).
 * warm = 1: each denoiser call starts from the previous call's final dual (the
 * warm-dual reading of the GAP and ADMM loops; the paper starts every call at
 * zero); warm = 0: every call starts at zero.
 * Returns x^(T) and theta^(T+1); -1 if every mask entry is zero (L = 0). */
int orc_fista_tv(int kind, int B, int nx, int ny, double lambda, int T, int N, int accel, int warm,
                 const double *Y, const double *C, const double *x_init, double *x_out, double *theta_out)
{
    size_t V = (size_t)B * nx * ny, n = (size_t)nx * ny;
    const double L = orc_lipschitz(B, nx, ny, C);
    if (!(L > 0.0)) return -1;
    double *P = (double *)calloc(2 * V, sizeof(double)); /* carried dual [2][V] (warm) */
    double *r = (double *)malloc(n * sizeof(double));
    double *cr = (double *)malloc(V * sizeof(double));
    double *th = (double *)malloc(V * sizeof(double));
    double *z = (double *)malloc(V * sizeof(double));
    double *x = (double *)malloc(V * sizeof(double));
    double *xp = (double *)malloc(V * sizeof(double));
    if (x_init) memcpy(th, x_init, V * sizeof(double));
    else orc_adjoint(B, nx, ny, C, Y, th);
    memcpy(x, th, V * sizeof(double)); /* x^(0) */
    double tau = 1.0;
    for (int t = 1; t <= T; ++t) {
        memcpy(xp, x, V * sizeof(double));
        grad_step(B, nx, ny, C, Y, 1.0 / L, th, r, cr, z);
        orc_tv_denoise(kind, B, nx, ny, lambda / L, N, accel, 0, 0, z, warm ? P : NULL, x, P, P + V);
        const double tau1 = (1.0 + sqrt(1.0 + 4.0 * tau * tau)) / 2.0;
        const double c = (tau - 1.0) / tau1;
        for (size_t k = 0; k < V; ++k) th[k] = x[k] + c * (x[k] - xp[k]);
        tau = tau1;
    }
    memcpy(x_out, x, V * sizeof(double));
    if (theta_out) memcpy(theta_out, th, V * sizeof(double));
    free(P); free(r); free(cr); free(th); free(z); free(x); free(xp);
    return 0;
}

/* TwIST (Sec. 2.2) for the same objective:
 *   x^(0) = Phi^T y (or x_init)
 *   z^(t)     = x^(t) + (1/L) Phi^T (y - Phi x^(t))   (the printed step 1 assumes
 *               Phi scaled to ||Phi|| <= 1; 1/L is that scaling)
 *   theta^(t) = TVdenoise(z^(t)) with weight lambda / L
 *   x^(1)     = theta^(0)  (one plain iterative-shrinkage step starts the
 *               two-step recursion, which needs x^(t-1))
 *   x^(t+1)   = (1 - alpha) x^(t-1) + (alpha - beta) x^(t) + beta theta^(t),  t >= 1
 * warm as for FISTA.
 * Returns x^(T) and theta^(T-1) (the last denoiser output; x^(0) when T = 0);
 * -1 if L = 0. */
int orc_twist_tv(int kind, int B, int nx, int ny, double lambda, double alpha, double beta, int T, int N, int accel,
                 int warm, const double *Y, const double *C, const double *x_init, double *x_out, double *theta_out)
{
    size_t V = (size_t)B * nx * ny, n = (size_t)nx * ny;
    const double L = orc_lipschitz(B, nx, ny, C);
    if (!(L > 0.0)) return -1;
    double *P = (double *)calloc(2 * V, sizeof(double)); /* carried dual [2][V] (warm) */
    double *r = (double *)malloc(n * sizeof(double));
    double *cr = (double *)malloc(V * sizeof(double));
    double *th = (double *)malloc(V * sizeof(double));
    double *z = (double *)malloc(V * sizeof(double));
    double *x = (double *)malloc(V * sizeof(double));
    double *xp = (double *)malloc(V * sizeof(double));
    if (x_init) memcpy(x, x_init, V * sizeof(double));
    else orc_adjoint(B, nx, ny, C, Y, x);
    memcpy(th, x, V * sizeof(double));
    for (int t = 0; t < T; ++t) {
        grad_step(B, nx, ny, C, Y, 1.0 / L, x, r, cr, z);
        orc_tv_denoise(kind, B, nx, ny, lambda / L, N, accel, 0, 0, z, warm ? P : NULL, th, P, P + V);
        if (t == 0) {
            memcpy(xp, x, V * sizeof(double));
            memcpy(x, th, V * sizeof(double));
        } else {
            for (size_t k = 0; k < V; ++k) {
                const double xn = (1.0 - alpha) * xp[k] + (alpha - beta) * x[k] + beta * th[k];
                xp[k] = x[k];
                x[k] = xn;
            }
        }
    }
    memcpy(x_out, x, V * sizeof(double));
    if (theta_out) memcpy(theta_out, th, V * sizeof(double));
    free(P); free(r); free(cr); free(th); free(z); free(x); free(xp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Metrics.                                                                 */
/* ------------------------------------------------------------------------ */

/* PSNR = 10 log10(peak^2 / MSE), MSE over all `count` elements. */
double orc_psnr(long count, const double *a, const double *ref, double peak)
{
    double se = 0.0;
    for (long c = 0; c < count; ++c) se += (a[c] - ref[c]) * (a[c] - ref[c]);
    double mse = se / (double)count;
    return 10.0 * log10(peak * peak / mse);
}

/* ||Y - Phi x||^2 */
double orc_residual_sq(int B, int nx, int ny, const double *C, const double *X, const double *Y)
{
    size_t n = (size_t)nx * ny;
    double *f = (double *)malloc(n * sizeof(double));
    orc_forward(B, nx, ny, C, X, f);
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += (Y[c] - f[c]) * (Y[c] - f[c]);
    free(f);
    return s;
}
